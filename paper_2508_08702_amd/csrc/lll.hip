// Steps 1-2 of Algorithm 1 (paper, Section 2) on the GPU: build the
// generator matrix of eq. (2) (binary case r_max = c_i = 1, scale N), reduce
// it with LLL, and extract the kernel lattice basis.
//
// One 64-lane wave per instance.  The basis b_0..b_n (int64, n+1 vectors of
// length m+n+1) lives in global memory; lane l always owns columns
// l, l+64, l+128, so row operations never need another lane's data.  The
// exact integer Gram matrix G (lower triangle, int64) and the Gram-Schmidt
// data (mu lower triangle, B_i = ||b*_i||^2, FP64) live in LDS.
//
// The LLL loop follows the textbook floating-point variant: the GS row of
// b_k is recomputed from the exact Gram entries (r_kj = G_kj - sum_{i<j}
// mu_ji r_ki, mu_kj = r_kj / B_j), b_k is size reduced against b_{k-1}..b_0
// with exact int64 updates of the basis and of G (b_k -= q b_j), the GS row
// is recomputed after any reduction until none is needed, and then the
// Lovász condition with parameter delta decides between a swap and k+1.
// Termination is guarded by an iteration cap; integers are guarded against
// overflow.  Afterwards the vectors whose first m entries are zero are kept in
// reduced order and written without those entries (step 2 of Algorithm 1).
#include "msp_internal.h"

namespace msp {

namespace {

constexpr int kLanes = 64;
constexpr int kMaxCols = 3;  // columns per lane: m + n + 1 <= 192

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }  // i >= j

__device__ __forceinline__ long long gram_at(const long long *G, int i, int j) {
    return i >= j ? G[tri(i, j)] : G[tri(j, i)];
}

// Broadcast of lane src's double to the whole wave (src uniform).
__device__ __forceinline__ double bcast(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

}  // namespace

__global__ void __launch_bounds__(kLanes) lll_kernel(LllArgs a) {
    const int inst = blockIdx.x;
    const size_t si = (size_t)inst * a.stride;  // 4-byte units
    const int m = a.m[si], n = a.n[si];
    const int nv = n + 1, len = m + n + 1;
    const int lane = threadIdx.x;
    const int64_t A_off = *reinterpret_cast<const int64_t *>(reinterpret_cast<const int32_t *>(a.A_off) + si);
    const int64_t d_off = *reinterpret_cast<const int64_t *>(reinterpret_cast<const int32_t *>(a.d_off) + si);
    const int64_t w_off = *reinterpret_cast<const int64_t *>(reinterpret_cast<const int32_t *>(a.work_off) + si);
    const int64_t o_off = *reinterpret_cast<const int64_t *>(reinterpret_cast<const int32_t *>(a.out_off) + si);
    long long *B = a.work + w_off;                       // nv x len
    int32_t *status = a.status + si;
    int32_t *kout = a.kout + si;
    long long *iters_out = reinterpret_cast<long long *>(reinterpret_cast<int32_t *>(a.iters) + si);
    extern __shared__ __align__(16) unsigned char smem[];
    long long *G = reinterpret_cast<long long *>(smem);  // nv(nv+1)/2
    double *mu = reinterpret_cast<double *>(G + nv * (nv + 1) / 2);  // nv(nv-1)/2, row k at k(k-1)/2
    double *Bn = mu + nv * (nv - 1) / 2;                 // nv
    double *rr = Bn + nv;                                // nv scratch: r_kj of the current row
    int *sflag = reinterpret_cast<int *>(rr + nv);       // [0] overflow

    const int32_t *A = a.A + A_off;
    const int64_t *d = a.d + d_off;
    const long long N = a.N;

    // ---- eq. (2): vector 0 = (-N d; -r_max x n; r_max), vector j = (N a_j; 2 c_j e_j; 0)
    // (binary variables: r_max = c_j = 1)
    const long long rm = a.cvec ? a.rmax : 1;
    for (int r = 0; r < nv; ++r) {
        for (int q = 0; q < kMaxCols; ++q) {
            const int c = lane + q * kLanes;
            if (c >= len) continue;
            long long v;
            if (r == 0)
                v = c < m ? -N * (long long)d[c] : (c < m + n ? -rm : rm);
            else
                v = c < m ? N * (long long)A[(size_t)c * n + (r - 1)]
                          : (c == m + (r - 1) ? 2 * (a.cvec ? (long long)a.cvec[r - 1] : 1) : 0);
            B[(size_t)r * len + c] = v;
        }
    }
    if (lane == 0) sflag[0] = 0;
    __syncthreads();
    // entries beyond 2^26 could overflow the exact int64 Gram products
    for (int r = 0; r < nv; ++r)
        for (int q = 0; q < kMaxCols; ++q) {
            const int c = lane + q * kLanes;
            if (c < len) {
                const long long v = B[(size_t)r * len + c];
                if (v > (1ll << 26) || v < -(1ll << 26)) sflag[0] = 1;
            }
        }
    __syncthreads();
    if (sflag[0]) {
        if (lane == 0) {
            status[0] = -4;
            kout[0] = 0;
            iters_out[0] = 0;
        }
        return;
    }
    // exact Gram matrix (lower triangle): |entries| < 192 * 2^52 < 2^60
    for (int e = lane; e < nv * (nv + 1) / 2; e += kLanes) {
        int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
        while (tri(i, 0) > e) --i;
        while (tri(i + 1, 0) <= e) ++i;
        const int j = e - tri(i, 0);
        long long s = 0;
        for (int c = 0; c < len; ++c) s += B[(size_t)i * len + c] * B[(size_t)j * len + c];
        G[e] = s;
    }
    __syncthreads();

    // GS row k from the exact Gram row, column by column (forward
    // substitution): r_ki = G_ki - sum_{j<i} mu_ij r_kj, mu_ki = r_ki / B_i.
    // Lane l keeps the running sum acc_l = sum_{j<i} mu_lj r_kj for its
    // columns l and l + 64; at column i the owner's r_ki is broadcast with a
    // readlane and every later column adds mu_li r_ki (a zero coefficient for
    // the others leaves their sums as they are).  The divisions and the sum
    // for B_k follow the loop, one per column in parallel.
    constexpr int kAhead = 8;
    auto gs_row = [&](int k) {
        const int j0 = lane, j1 = lane + 64;
        const double g0 = j0 < k ? (double)gram_at(G, k, j0) : 0.0;
        const double g1 = j1 < k ? (double)gram_at(G, k, j1) : 0.0;
        double acc0 = 0.0, acc1 = 0.0, r0 = 0.0, r1 = 0.0;
        for (int ib = 0; ib < k; ib += kAhead) {
            double c0[kAhead], c1[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                const int i = ib + u;
                const bool v0 = j0 > i && j0 < k, v1 = j1 > i && j1 < k;
                c0[u] = mu[v0 ? j0 * (j0 - 1) / 2 + i : 0];
                c1[u] = mu[v1 ? j1 * (j1 - 1) / 2 + i : 0];
                if (!v0) c0[u] = 0.0;
                if (!v1) c1[u] = 0.0;
            }
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                const int i = ib + u;
                if (i < k) {
                    double r;
                    if (i < 64) {
                        const double t = g0 - acc0;
                        if (lane == i) r0 = t;
                        r = bcast(t, i);
                    } else {
                        const double t = g1 - acc1;
                        if (lane == i - 64) r1 = t;
                        r = bcast(t, i - 64);
                    }
                    acc0 += c0[u] * r;
                    acc1 += c1[u] * r;
                }
            }
        }
        double s = 0.0;
        if (j0 < k) {
            const double mki = r0 / Bn[j0];
            mu[k * (k - 1) / 2 + j0] = mki;
            s += mki * r0;
        }
        if (j1 < k) {
            const double mki = r1 / Bn[j1];
            mu[k * (k - 1) / 2 + j1] = mki;
            s += mki * r1;
        }
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) Bn[k] = (double)gram_at(G, k, k) - s;
        __syncthreads();
    };

    // One pass of size reduction of b_k against b_{k-1}, ..., b_0: for j
    // descending, b_k -= rint(mu_kj) b_j wherever |mu_kj| > 0.51, with the mu
    // row updated after each subtraction (mu_ki -= q mu_ji for i < j, mu_kj -=
    // q).  The mu row is held in registers and the next column is the highest
    // one over the threshold, found by ballot; the multiples q_j are collected
    // and the basis row and the Gram row are updated once at the end:
    //   b_k' = b_k - sum_j q_j b_j,  G_ki' = G_ki - sum_j q_j G_ji (i != k),
    //   G_kk' = G_kk - sum_j q_j (G_kj + G_kj').
    // The new row's squared length, B_k + sum_i mu_ki'^2 B_i, bounds every
    // updated entry; while it is below 2^61 the exact values fit in int64 and
    // wrapping int64 arithmetic computes them exactly, and the exact diagonal
    // entry is then checked against the estimate and against 2^62.  Returns
    // whether anything was subtracted; sets st = -10 for a multiple beyond the
    // exact integer range.
    auto reduce_pass = [&](int k, int &stat) -> bool {
        const int j0 = lane, j1 = lane + 64;
        const int rk = k * (k - 1) / 2;
        double m0 = j0 < k ? mu[rk + j0] : 0.0;
        double m1 = j1 < k ? mu[rk + j1] : 0.0;
        long long q0 = 0, q1 = 0;
        int top = k;
        for (;;) {
            const unsigned long long b1 = __ballot(j1 < top && !(fabs(m1) <= 0.51));
            const unsigned long long b0 = __ballot(j0 < top && !(fabs(m0) <= 0.51));
            int j;
            double mj;
            if (b1) {
                j = 64 + 63 - __clzll(b1);
                mj = bcast(m1, j - 64);
            } else if (b0) {
                j = 63 - __clzll(b0);
                mj = bcast(m0, j);
            } else {
                break;
            }
            if (!(fabs(mj) < 9.0e15)) {  // NaN or beyond exact integer range
                stat = -10;
                return true;
            }
            const long long q = (long long)rint(mj);
            const double qd = (double)q;
            const int rj = j * (j - 1) / 2;
            if (j0 < j) m0 -= qd * mu[rj + j0];
            if (j1 < j) m1 -= qd * mu[rj + j1];
            if (j0 == j) m0 -= qd, q0 = q;
            if (j1 == j) m1 -= qd, q1 = q;
            top = j;
        }
        if (top == k) return false;
        // basis row (global memory; lane owns columns lane + 64 t) and Gram row
        uint64_t bk[kMaxCols];
#pragma unroll
        for (int c4 = 0; c4 < kMaxCols; ++c4) {
            const int c = lane + c4 * kLanes;
            bk[c4] = c < len ? (uint64_t)B[(size_t)k * len + c] : 0;
        }
        for (int h = 0; h < 2; ++h) {
            unsigned long long nz = __ballot((h ? q1 : q0) != 0);
            while (nz) {
                const int bit = __ffsll(nz) - 1;
                nz &= nz - 1;
                const int j = bit + h * 64;
                const long long qv = h ? q1 : q0;
                const uint64_t q = ((uint64_t)(unsigned)__builtin_amdgcn_readlane((int)(qv >> 32), bit) << 32) |
                                   (unsigned)__builtin_amdgcn_readlane((int)qv, bit);
#pragma unroll
                for (int c4 = 0; c4 < kMaxCols; ++c4) {
                    const int c = lane + c4 * kLanes;
                    if (c < len) bk[c4] -= q * (uint64_t)B[(size_t)j * len + c];
                }
            }
        }
        double est = 0.0;
        if (j0 < k) est = m0 * m0 * Bn[j0];
        if (j1 < k) est += m1 * m1 * Bn[j1];
        for (int o = 32; o >= 1; o >>= 1) est += __shfl_xor(est, o, 64);
        est += Bn[k];
        bool bad = !(est < 0x1p61);
        uint64_t gold[2], gnew[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = lane + h * 64;
            gold[h] = (i < nv && i != k) ? (uint64_t)gram_at(G, k, i) : 0;
            gnew[h] = gold[h];
        }
        for (int h = 0; h < 2; ++h) {
            unsigned long long nz = __ballot((h ? q1 : q0) != 0);
            while (nz) {
                const int bit = __ffsll(nz) - 1;
                nz &= nz - 1;
                const int j = bit + h * 64;
                const long long qv = h ? q1 : q0;
                const uint64_t q = ((uint64_t)(unsigned)__builtin_amdgcn_readlane((int)(qv >> 32), bit) << 32) |
                                   (unsigned)__builtin_amdgcn_readlane((int)qv, bit);
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    const int i = lane + g * 64;
                    const uint64_t gj = (uint64_t)gram_at(G, j, i < nv ? i : 0);
                    if (i < nv && i != k) gnew[g] -= q * gj;
                }
            }
        }
        uint64_t dsum = 0;
        if (q0) dsum += (uint64_t)q0 * (gold[0] + gnew[0]);
        if (q1) dsum += (uint64_t)q1 * (gold[1] + gnew[1]);
        for (int o = 32; o >= 1; o >>= 1) dsum += (uint64_t)__shfl_xor((long long)dsum, o, 64);
        const long long nd = (long long)((uint64_t)gram_at(G, k, k) - dsum);
        if (nd <= 0 || nd > (1ll << 62) || fabs((double)nd - est) > 0.5 * est + 1024.0) bad = true;
        __syncthreads();
#pragma unroll
        for (int c4 = 0; c4 < kMaxCols; ++c4) {
            const int c = lane + c4 * kLanes;
            if (c < len) B[(size_t)k * len + c] = (long long)bk[c4];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = lane + h * 64;
            if (i < nv && i != k) G[i >= k ? tri(i, k) : tri(k, i)] = (long long)gnew[h];
            if (i < k) mu[rk + i] = h ? m1 : m0;
        }
        if (lane == 0) G[tri(k, k)] = nd;
        if (__ballot(bad) && lane == 0) sflag[0] = 1;
        __syncthreads();
        return true;
    };

    if (lane == 0) Bn[0] = (double)G[0];
    __syncthreads();
    int k = 1;
    long long iters = 0;
    int st = 0;
    const double delta = a.delta;
    while (k < nv) {
        if (++iters > a.max_iters) {
            st = -10;  // no convergence
            break;
        }
        gs_row(k);
        // lazy size reduction: reduce, recompute the GS row, until stable
        for (int round = 0; round < 64; ++round) {
            if (!reduce_pass(k, st)) break;
            if (st) break;
            gs_row(k);
        }
        if (st) break;
        if (sflag[0]) {
            st = -4;
            break;
        }
        const double mk = mu[k * (k - 1) / 2 + (k - 1)];
        if (delta * Bn[k - 1] > Bn[k] + mk * mk * Bn[k - 1]) {
            // swap b_{k-1} and b_k: basis rows and Gram rows/columns
            for (int c4 = 0; c4 < kMaxCols; ++c4) {
                const int c = lane + c4 * kLanes;
                if (c >= len) continue;
                const long long t0 = B[(size_t)(k - 1) * len + c];
                B[(size_t)(k - 1) * len + c] = B[(size_t)k * len + c];
                B[(size_t)k * len + c] = t0;
            }
            long long g0a = 0, g0b = 0, g1a = 0, g1b = 0;
            const int i0 = lane, i1 = lane + 64;
            if (i0 < nv && i0 != k && i0 != k - 1) { g0a = gram_at(G, k - 1, i0); g0b = gram_at(G, k, i0); }
            if (i1 < nv && i1 != k && i1 != k - 1) { g1a = gram_at(G, k - 1, i1); g1b = gram_at(G, k, i1); }
            const long long dkk = gram_at(G, k, k), dk1 = gram_at(G, k - 1, k - 1);
            __syncthreads();
            auto put = [&](int r, int i, long long v) { G[r >= i ? tri(r, i) : tri(i, r)] = v; };
            if (i0 < nv && i0 != k && i0 != k - 1) { put(k - 1, i0, g0b); put(k, i0, g0a); }
            if (i1 < nv && i1 != k && i1 != k - 1) { put(k - 1, i1, g1b); put(k, i1, g1a); }
            if (lane == 0) { put(k, k, dk1); put(k - 1, k - 1, dkk); }
            __syncthreads();
            if (k - 1 == 0) {
                if (lane == 0) Bn[0] = (double)G[0];
                __syncthreads();
            }
            k = k - 1 > 1 ? k - 1 : 1;  // rows below k are unchanged; row k is recomputed next
        } else {
            ++k;
        }
    }
    if (st == 0 && sflag[0]) st = -4;

    // ---- step 2: keep the zero-top vectors in reduced order
    int count = 0;
    if (st == 0) {
        const int kexp = n - m + 1;
        for (int r = 0; r < nv; ++r) {
            bool zero = true;
            for (int c4 = 0; c4 < kMaxCols; ++c4) {
                const int c = lane + c4 * kLanes;
                if (c < m && B[(size_t)r * len + c] != 0) zero = false;
            }
            const bool allzero = __ballot(!zero) == 0;
            if (allzero) {
                if (count < kexp) {
                    int64_t *out = a.out + o_off + (size_t)count * (n + 1);
                    for (int c4 = 0; c4 < kMaxCols; ++c4) {
                        const int c = lane + c4 * kLanes;
                        if (c >= m && c < len) out[c - m] = B[(size_t)r * len + c];
                    }
                }
                ++count;
            }
        }
        if (count < kexp) st = -3;
        else if (count > kexp) st = -2;
    }
    if (lane == 0) {
        status[0] = st;
        kout[0] = count;
        iters_out[0] = iters;
    }
}

size_t lll_lds_bytes(int n) {
    const size_t nv = (size_t)n + 1;
    return nv * (nv + 1) / 2 * sizeof(long long) + nv * (nv - 1) / 2 * sizeof(double) +
           2 * nv * sizeof(double) + 16;
}

hipError_t launch_lll(const LllArgs &a, int ninst, int max_n, hipStream_t st) {
    const size_t lds = lll_lds_bytes(max_n);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)lll_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lll_kernel, dim3(ninst), dim3(kLanes), lds, st, a);
    return hipGetLastError();
}

__global__ void bounds_scale_kernel(const int32_t *r, int n, int64_t *cvec, long long *rmax) {
    if (threadIdx.x != 0) return;
    long long l = 1;
    bool bad = false;
    for (int j = 0; j < n && !bad; ++j) {
        const long long v = r[j];
        if (v < 1 || v > 255) {
            *rmax = -1;
            return;
        }
        long long g = l, h = v;
        while (h) {
            const long long t = g % h;
            g = h;
            h = t;
        }
        l = l / g * v;
        if (l > (1ll << 20)) bad = true;
    }
    if (!bad)
        for (int j = 0; j < n; ++j) cvec[j] = l / r[j];
    *rmax = bad ? -2 : l;
}

hipError_t launch_bounds_scale(const int32_t *r, int n, int64_t *cvec, long long *rmax, hipStream_t st) {
    hipLaunchKernelGGL(bounds_scale_kernel, dim3(1), dim3(64), 0, st, r, n, cvec, rmax);
    return hipGetLastError();
}

}  // namespace msp
