// Per-level rules of the enumeration (paper, Section 2 and Algorithm 1),
// shared by the root generator and the subtree walker.
//
// Centre and partial norm are evaluated with every product and sum rounded
// on its own (no fused multiply-add), in a fixed order, so that these scalar
// recurrences -- which decide the l2 pruning -- are reproducible bit for bit:
//   y_t = sum_{i>t} u_i mu_{i,t}   (centre c_t = -y_t): term p = k-1-i (p = 0
//         is the top level) goes to partial sum s_(p mod 8), each partial
//         sum runs from the top level down starting at 0, and
//         y_t = ((s0 + s1) + (s2 + s3)) + ((s4 + s5) + (s6 + s7));
//   l   = (x * x) * beta_t + l'   (x = u_t + y_t)
// Eight interleaved sums make the dependent chain eight times shorter than
// one running sum; any fixed order serves, as long as it is the same
// everywhere.
#pragma once

#include <hip/hip_runtime.h>

namespace msp {

#pragma clang fp contract(off)

__device__ __forceinline__ double add_rn(double a, double b) { return a + b; }
__device__ __forceinline__ double mul_rn(double a, double b) { return a * b; }

__device__ __forceinline__ double partial_norm(double x, double beta, double lpar) {
    return add_rn(mul_rn(mul_rn(x, x), beta), lpar);
}

__device__ __forceinline__ double combine8(const double (&s)[8]) {
    return add_rn(add_rn(add_rn(s[0], s[1]), add_rn(s[2], s[3])), add_rn(add_rn(s[4], s[5]), add_rn(s[6], s[7])));
}

// Centre sum for a prefix in natural level order (u[i] = u_i) and mu row-major
// (mu[i * k + t] = mu_{i,t}).
__device__ __forceinline__ double centre_natural(const int8_t *u, const double *mu, int k, int t) {
    double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const int nt = k - 1 - t;
    for (int p0 = 0; p0 < nt; p0 += 8) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int p = p0 + r;
            if (p < nt) {
                const int i = k - 1 - p;
                s[r] = add_rn(s[r], mul_rn((double)u[i], mu[(size_t)i * k + t]));
            }
        }
    }
    return combine8(s);
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

// Direction kept after the first Hoelder failure: the side of c that u is on.
__device__ __forceinline__ int side_of(int u, double y) { return add_rn((double)u, y) > 0.0 ? 1 : -1; }

#pragma clang fp contract(fast)

}  // namespace msp
