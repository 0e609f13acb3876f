// Root generation over thin levels in one launch (see expand_thin_kernel).
#pragma once

#include "msp_internal.h"

namespace msp {

constexpr int kThinBlock = 1024;                   // one workgroup
constexpr int kThinPer = 1;                        // parents per thread and level
constexpr int kThinMax = kThinBlock * kThinPer;    // most parents a thin level takes

// When root generation stops, as a function of the frontier (n nodes at
// level L):  kind 0: k - L >= depth (a fixed split depth);  kind 1: n >= target
// and L <= lb (the automatic split);  kind 2: n >= target or L <= lb (the
// refinement stages of an ordered first-solution search).
struct ThinRule {
    int kind;
    int k, depth, lb;
    int64_t target;
};

__host__ __device__ inline bool thin_done(const ThinRule &r, int64_t n, int L) {
    if (r.kind == 0) return r.k - L >= r.depth;
    if (r.kind == 1) return n >= r.target && L <= r.lb;
    return n >= r.target || L <= r.lb;
}

struct ThinOut {
    int64_t np;  // nodes of the last level taken
    int L;       // its level
    int cur;     // the frontier buffer that holds it (index into ThinArgs::fr)
    int capped;  // 1: the next level would not have fit the buffers
    int pad;
};

struct ThinArgs {
    ExpandArgs e;    // the per-level arguments (t, par, ch, np, offs, counts unused)
    Frontier fr[2];  // fr[0]: the np parents at level L; fr[1]: the other buffer
    int64_t np;      // 1 .. kThinMax
    int L;
    int64_t fcap;    // frontier buffer capacity (records)
    ThinRule rule;
    ThinOut *out;    // device memory
};

hipError_t launch_expand_thin(const ThinArgs &a, hipStream_t st);

}  // namespace msp
