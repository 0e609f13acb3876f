// Per-level rules of the enumeration (paper, Section 2 and Algorithm 1),
// shared by the root generator and the subtree walker.
//
// Centre and partial norm are evaluated with every product and sum rounded
// on its own (no fused multiply-add), in a fixed order, so that these scalar
// recurrences -- which decide the l2 pruning -- are reproducible bit for bit:
//   y_t = sum_{i = k-1 down to t+1} u_i mu_{i,t}     (centre c_t = -y_t)
//   l   = (x * x) * beta_t + l'                       (x = u_t + y_t)
#pragma once

#include <hip/hip_runtime.h>

namespace msp {

#pragma clang fp contract(off)

__device__ __forceinline__ double add_rn(double a, double b) { return a + b; }
__device__ __forceinline__ double mul_rn(double a, double b) { return a * b; }

__device__ __forceinline__ double partial_norm(double x, double beta, double lpar) {
    return add_rn(mul_rn(mul_rn(x, x), beta), lpar);
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

// Direction kept after the first Hoelder failure: the side of c that u is on.
__device__ __forceinline__ int side_of(int u, double y) { return add_rn((double)u, y) > 0.0 ? 1 : -1; }

#pragma clang fp contract(fast)

}  // namespace msp
