// Per-level rules of the enumeration (paper, Section 2 and Algorithm 1),
// shared by the root generator, the root features and the subtree walker.
//
// Centre and partial norm are evaluated in one fixed order everywhere on the
// GPU, so that every kernel that meets the same prefix takes the same pruning
// decisions (the split level and the dynamic splitting of the walk then do
// not change the search-tree counters):
//   y_t = sum_{i>t} u_i mu_{i,t}   (centre c_t = -y_t): term p = k-1-i (p = 0
//         is the top level) goes to partial sum s_(p mod 4); each partial sum
//         runs from the top level down, starting at 0, with fused
//         multiply-adds, and y_t = (s0 + s1) + (s2 + s3);
//   l   = fma(x * x, beta_t, l')   (x = u_t + y_t).
// Four interleaved sums keep the dependent chain short.  The order differs
// from the plain sum the paper writes only in rounding, far below the 1e-9
// slack of the pruning tests.
#pragma once

#include <hip/hip_runtime.h>

namespace msp {

#pragma clang fp contract(off)

__device__ __forceinline__ double add_rn(double a, double b) { return a + b; }
__device__ __forceinline__ double mul_rn(double a, double b) { return a * b; }

__device__ __forceinline__ double partial_norm(double x, double beta, double lpar) {
    return fma(mul_rn(x, x), beta, lpar);
}

__device__ __forceinline__ double combine4(double s0, double s1, double s2, double s3) {
    return add_rn(add_rn(s0, s1), add_rn(s2, s3));
}

// Centre sum for a prefix in natural level order (u[i] = u_i) and mu row-major
// (mu[i * k + t] = mu_{i,t}).
__device__ __forceinline__ double centre_natural(const int8_t *u, const double *mu, int k, int t) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    const int nt = k - 1 - t;
    for (int p0 = 0; p0 < nt; p0 += 4) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int p = p0 + r;
            if (p < nt) {
                const int i = k - 1 - p;
                s[r] = fma((double)u[i], mu[(size_t)i * k + t], s[r]);
            }
        }
    }
    return combine4(s[0], s[1], s[2], s[3]);
}

// Zig-zag state of one level: values u1, u1+s, u1-s, u1+2s, ... around the
// centre c = -y (Algorithm 1, next()); u1 = rint(c) (ties to even) and the
// first step s goes to the other side of c (s = +1 when u1 - c <= 0).
// While every u above the level is zero the sign symmetry v <-> -v is broken
// by trying only 0, 1, 2, ... (one direction from the start).
struct Zig {
    int u1, s;
};

__device__ __forceinline__ Zig zig_init(double y, bool topzero) {
    Zig z;
    if (topzero) {
        z.u1 = 0;
        z.s = 1;
    } else {
        const double c = -y;
        z.u1 = (int)rint(c);
        z.s = (add_rn((double)z.u1, -c) <= 0.0) ? 1 : -1;
    }
    return z;
}

// Next value after u in the zig-zag sequence.
__device__ __forceinline__ int zig_next(const Zig &z, int u) {
    const int o = u - z.u1;
    int no;
    if (o == 0)
        no = z.s;
    else if ((o > 0) == (z.s > 0))
        no = -o;
    else
        no = -o + z.s;
    return z.u1 + no;
}

// Rank of u in the level's value order (limited discrepancy search, Section 3:
// the discrepancy cost of taking u): u on a top-zero level, else 0 for u1 and
// 2|o|-1 or 2|o| for u1 + o on the side of s or the other side.  Ranks never
// decrease along a level, one-direction runs included.
__device__ __forceinline__ int zig_rank(const Zig &z, int u, bool topzero) {
    if (topzero) return u;
    const int o = u - z.u1;
    if (o == 0) return 0;
    const int ao = o < 0 ? -o : o;
    return ((o > 0) == (z.s > 0)) ? 2 * ao - 1 : 2 * ao;
}

// Discrepancy cost of taking u (limited discrepancy search, Section 3): its
// rank (reading "rank"), or 1 for every value but the level's first (reading
// "count": the number of departures from the heuristic's choice).  Under
// both readings the cost never decreases along a level.
__device__ __forceinline__ int disc_cost(const Zig &z, int u, bool topzero, bool count) {
    const int r = zig_rank(z, u, topzero);
    return count ? (r > 0 ? 1 : 0) : r;
}

// Direction kept after the first Hoelder failure: the side of c that u is on.
__device__ __forceinline__ int side_of(int u, double y) { return add_rn((double)u, y) > 0.0 ? 1 : -1; }

#pragma clang fp contract(fast)

}  // namespace msp
