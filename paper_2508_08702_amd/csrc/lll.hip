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

    // GS row k from the exact Gram row (forward substitution, lanes own j)
    auto gs_row = [&](int k) {
        double acc0 = 0.0, acc1 = 0.0;  // sum_{i<j} mu_ji r_ki for j = lane, lane + 64
        for (int i = 0; i < k; ++i) {
            const int owner = i & 63;
            double r = 0.0;
            if (lane == owner) r = (double)gram_at(G, k, i) - (i < 64 ? acc0 : acc1);
            r = __shfl(r, owner, 64);
            const double mki = r / Bn[i];
            if (lane == 0) {
                rr[i] = r;
                mu[k * (k - 1) / 2 + i] = mki;
            }
            const int j0 = lane, j1 = lane + 64;
            if (j0 > i && j0 < k) acc0 += mu[j0 * (j0 - 1) / 2 + i] * r;
            if (j1 > i && j1 < k) acc1 += mu[j1 * (j1 - 1) / 2 + i] * r;
        }
        __syncthreads();
        double s = 0.0;
        for (int i = lane; i < k; i += 64) s += mu[k * (k - 1) / 2 + i] * rr[i];
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) Bn[k] = (double)gram_at(G, k, k) - s;
        __syncthreads();
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
            bool any = false;
            for (int j = k - 1; j >= 0; --j) {
                const double mkj = mu[k * (k - 1) / 2 + j];
                if (!(fabs(mkj) <= 0.51)) {
                    if (!(fabs(mkj) < 9.0e15)) {  // NaN or beyond exact integer range
                        st = -10;
                        break;
                    }
                    const long long q = (long long)rint(mkj);
                    any = true;
                    const double qa = fabs((double)q);
                    // basis row: b_k -= q b_j (exact; magnitudes estimated first)
                    for (int c4 = 0; c4 < kMaxCols; ++c4) {
                        const int c = lane + c4 * kLanes;
                        if (c >= len) continue;
                        const long long bj = B[(size_t)j * len + c];
                        if (qa * fabs((double)bj) > 1.0e15) {
                            sflag[0] = 1;
                            continue;
                        }
                        const long long nvv = B[(size_t)k * len + c] - q * bj;
                        if (nvv > (1ll << 50) || nvv < -(1ll << 50)) sflag[0] = 1;
                        B[(size_t)k * len + c] = nvv;
                    }
                    // Gram: G_kk' = G_kk - 2q G_kj + q^2 G_jj, G_ki' = G_ki - q G_ji (i != k);
                    // every lane reads the old values before any lane writes
                    const long long gkj = gram_at(G, k, j), gjj = gram_at(G, j, j), gkk = gram_at(G, k, k);
                    const double est = fabs((double)gkk) + 2.0 * qa * fabs((double)gkj) + qa * qa * fabs((double)gjj);
                    if (est > 4.0e18) sflag[0] = 1;
                    long long newv0 = 0, newv1 = 0;
                    const int i0 = lane, i1 = lane + 64;
                    if (i0 < nv && i0 != k) {
                        const long long gji = gram_at(G, j, i0);
                        if (qa * fabs((double)gji) > 4.0e18) sflag[0] = 1;
                        newv0 = gram_at(G, k, i0) - q * gji;
                    }
                    if (i1 < nv && i1 != k) {
                        const long long gji = gram_at(G, j, i1);
                        if (qa * fabs((double)gji) > 4.0e18) sflag[0] = 1;
                        newv1 = gram_at(G, k, i1) - q * gji;
                    }
                    __syncthreads();
                    if (i0 < nv && i0 != k) G[i0 >= k ? tri(i0, k) : tri(k, i0)] = newv0;
                    if (i1 < nv && i1 != k) G[i1 >= k ? tri(i1, k) : tri(k, i1)] = newv1;
                    if (lane == 0 && est <= 4.0e18) G[tri(k, k)] = gkk - 2 * q * gkj + q * q * gjj;
                    // mu row k: mu_ki -= q mu_ji (i < j), mu_kj -= q
                    const double qd = (double)q;
                    for (int i = lane; i < j; i += 64) mu[k * (k - 1) / 2 + i] -= qd * mu[j * (j - 1) / 2 + i];
                    if (lane == 0) mu[k * (k - 1) / 2 + j] -= qd;
                    __syncthreads();
                }
            }
            if (st) break;
            if (!any) break;
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
