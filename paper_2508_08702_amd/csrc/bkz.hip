// Block Korkine-Zolotarev reduction of the kernel basis (paper, Section 2:
// the reduction step may use BKZ instead of LLL).  A better reduced basis
// leaves the solution set unchanged and shrinks the enumeration tree.
//
// One 64-lane wave per instance works on the k x dim int64 kernel basis in
// place.  The exact int64 Gram matrix (lower triangle) and the FP64
// Gram-Schmidt data (mu, beta) live in LDS.  A tour visits every block
// [j, h], h = min(j + beta, k) - 1:
//   * lane 0 finds a shortest nonzero vector of the block's projected
//     lattice by Schnorr-Euchner enumeration (radius 0.999 beta_j, shrunk to
//     each shorter vector found, node cap per block);
//   * if it is shorter than b*_j, it is inserted at position j by unimodular
//     row operations on b_j..b_h (integer, exact), and the basis is
//     LLL-reduced again from j;
// and tours repeat until one inserts nothing or the tour limit is reached.
#include "msp_internal.h"

namespace msp {

namespace {

constexpr int kW = 64;

__device__ __forceinline__ int tri(int i, int j) { return i * (i + 1) / 2 + j; }  // i >= j
__device__ __forceinline__ int trs(int i, int j) { return i * (i - 1) / 2 + j; }  // i > j (mu)

struct Bkz {
    int k, dim;
    int64_t *B;        // k x dim (global)
    long long *G;      // Gram, lower triangle (LDS)
    double *mu;        // mu_{ij}, i > j (LDS)
    double *bb;        // beta_i = ||b*_i||^2 (LDS)
    double *r;         // scratch row (LDS)
    int *flag;         // [0] overflow (LDS)
    int lane;

    __device__ long long gram(int i, int j) const { return i >= j ? G[tri(i, j)] : G[tri(j, i)]; }

    // Gram row i (all j) from the basis rows
    __device__ void gram_row(int i) {
        for (int j = lane; j < k; j += kW) {
            long long s = 0;
            for (int c = 0; c < dim; ++c) s += B[(size_t)i * dim + c] * B[(size_t)j * dim + c];
            if (j <= i)
                G[tri(i, j)] = s;
            else
                G[tri(j, i)] = s;
        }
        __syncthreads();
    }

    __device__ void gram_all() {
        for (int e = lane; e < k * (k + 1) / 2; e += kW) {
            int i = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
            while (tri(i, 0) > e) --i;
            while (tri(i + 1, 0) <= e) ++i;
            const int j = e - tri(i, 0);
            long long s = 0;
            for (int c = 0; c < dim; ++c) s += B[(size_t)i * dim + c] * B[(size_t)j * dim + c];
            G[e] = s;
        }
        __syncthreads();
    }

    // Gram-Schmidt row i from the exact Gram row and rows < i:
    // r_j = G_ij - sum_{l<j} mu_jl r_l, mu_ij = r_j / beta_j, beta_i = G_ii -
    // sum_j mu_ij r_j.  The sums are split over the lanes (lane l keeps r_j
    // for j = l mod 64 in r[]) and reduced across the wave.
    __device__ void gs_row(int i) {
        double rr_part = 0.0;
        for (int j = 0; j < i; ++j) {
            double part = 0.0;
            for (int l = lane; l < j; l += kW) part += mu[trs(j, l)] * r[l];
            for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, kW);
            const double s = (double)gram(i, j) - part;
            const double m = s / bb[j];
            if (lane == (j & (kW - 1))) {
                r[j] = s;
                mu[trs(i, j)] = m;
                rr_part += m * s;
            }
            __syncthreads();
        }
        for (int o = 32; o >= 1; o >>= 1) rr_part += __shfl_xor(rr_part, o, kW);
        if (lane == 0) bb[i] = (double)gram(i, i) - rr_part;
        __syncthreads();
    }

    // b_i -= q b_j for the basis, its Gram row/column i and mu row i
    __device__ void sub_row(int i, int j, long long q) {
        for (int c = lane; c < dim; c += kW) {
            const int64_t v = B[(size_t)i * dim + c] - q * B[(size_t)j * dim + c];
            if (v > (1ll << 26) || v < -(1ll << 26)) flag[0] = 1;  // keeps the Gram exact in int64
            B[(size_t)i * dim + c] = v;
        }
        __syncthreads();
        if (lane == 0)
            for (int l = 0; l < j; ++l) mu[trs(i, l)] -= (double)q * mu[trs(j, l)];
        if (lane == 0) mu[trs(i, j)] -= (double)q;
        __syncthreads();
        gram_row(i);
    }

    __device__ void swap_rows(int i, int j) {
        for (int c = lane; c < dim; c += kW) {
            const int64_t t = B[(size_t)i * dim + c];
            B[(size_t)i * dim + c] = B[(size_t)j * dim + c];
            B[(size_t)j * dim + c] = t;
        }
        __syncthreads();
    }

    // LLL (Lovasz delta) assuming rows < start have valid GS data
    __device__ void lll(int start, double delta, long long &budget) {
        int i = start < 1 ? 1 : start;
        if (start <= 0) gs_row(0);
        while (i < k && budget > 0 && !flag[0]) {
            --budget;
            gs_row(i);
            for (int j = i - 1; j >= 0; --j) {
                const double m = mu[trs(i, j)];
                if (fabs(m) > 0.51) {
                    const long long q = (long long)rint(m);
                    sub_row(i, j, q);
                }
            }
            gs_row(i);
            const double m1 = mu[trs(i, i - 1)];
            if (bb[i] >= (delta - m1 * m1) * bb[i - 1]) {
                ++i;
            } else {
                swap_rows(i - 1, i);
                gram_row(i - 1);
                gram_row(i);
                i = i - 1 > 1 ? i - 1 : 1;
                gs_row(i - 1);
            }
        }
    }
};

}  // namespace

__global__ void __launch_bounds__(kW) bkz_kernel(BkzArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int k = a.k, dim = a.dim, inst = blockIdx.x;
    int64_t *Bg = a.B + (size_t)inst * a.bstride;
    Bkz z;
    z.k = k;
    z.dim = dim;
    z.B = Bg;
    z.lane = threadIdx.x;
    z.G = reinterpret_cast<long long *>(smem);
    z.mu = reinterpret_cast<double *>(z.G + k * (k + 1) / 2);
    z.bb = z.mu + k * (k - 1) / 2 + 1;
    z.r = z.bb + k;
    int *x = reinterpret_cast<int *>(z.r + k);   // block coefficients (best)
    int *xc = x + k;                             // current coefficients
    z.flag = xc + k;
    double *cl = reinterpret_cast<double *>(z.flag + 2);  // per-level partial norms (k + 1)
    double *cc = cl + k + 1;                               // per-level centres
    int *st = reinterpret_cast<int *>(cc + k);             // per-level zig-zag state: u1, step count
    if (z.lane == 0) z.flag[0] = 0;
    // the basis itself in LDS when it fits (copied back at the end)
    int64_t *Bs = reinterpret_cast<int64_t *>(st + 2 * k);  // 8-byte aligned: st follows doubles
    if (a.b_in_lds) {
        for (int e = z.lane; e < k * dim; e += kW) Bs[e] = Bg[e];
        z.B = Bs;
    }
    __syncthreads();
    long long budget = a.max_lll_iters;
    z.gram_all();
    z.lll(0, a.delta, budget);
    long long inserted = 0, nodes_total = 0;
    for (int tour = 0; tour < a.tours && !z.flag[0] && budget > 0; ++tour) {
        int changed = 0;
        for (int j = 0; j + 1 < k && !z.flag[0] && budget > 0; ++j) {
            const int h = (j + a.beta < k ? j + a.beta : k) - 1;
            const int n = h - j + 1;
            // ---- block SVP by lane 0 ----
            // Schnorr-Euchner enumeration of the projected block lattice:
            // level t (0 = block start j) takes values in zig-zag order
            // around its centre, so the first value beyond the radius ends the
            // level; while every coefficient above is zero only 0, 1, 2, ...
            // are taken (v and -v are the same vector).
            int found = 0;
            if (z.lane == 0) {
                double R = z.bb[j] * 0.999;
                long long nodes = 0;
                for (int t = 0; t < n; ++t) {
                    xc[t] = 0;
                    x[t] = 0;
                }
                cl[n] = 0.0;
                int t = n - 1;
                cc[t] = 0.0;
                st[2 * t] = 0;
                st[2 * t + 1] = 1;  // top-zero level
                while (nodes < a.max_nodes) {
                    ++nodes;
                    const double dx = (double)xc[t] - cc[t];
                    const double l = dx * dx * z.bb[j + t] + cl[t + 1];
                    if (l < R) {
                        if (t > 0) {
                            cl[t] = l;
                            --t;
                            double c = 0.0;
                            int tz = 1;
                            for (int s2 = t + 1; s2 < n; ++s2) {
                                c -= (double)xc[s2] * z.mu[trs(j + s2, j + t)];
                                if (xc[s2]) tz = 0;
                            }
                            cc[t] = c;
                            st[2 * t + 1] = tz;
                            st[2 * t] = tz ? 0 : (int)rint(c);
                            xc[t] = st[2 * t];
                            continue;
                        }
                        bool nz = false;
                        for (int s2 = 0; s2 < n; ++s2)
                            if (xc[s2]) nz = true;
                        if (nz) {
                            R = l;
                            for (int s2 = 0; s2 < n; ++s2) x[s2] = xc[s2];
                            found = 1;
                        }
                    } else {
                        xc[t] = 0;
                        ++t;
                        if (t >= n) break;
                    }
                    // next value of level t
                    if (st[2 * t + 1]) {
                        xc[t] += 1;
                    } else {
                        const int u1 = st[2 * t];
                        const int s0 = ((double)u1 - cc[t] <= 0.0) ? 1 : -1;
                        const int off = xc[t] - u1;
                        int no;
                        if (off == 0)
                            no = s0;
                        else if ((off > 0) == (s0 > 0))
                            no = -off;
                        else
                            no = -off + s0;
                        xc[t] = u1 + no;
                    }
                }
                nodes_total += nodes;
            }
            found = __shfl(found, 0, kW);
            if (!found) continue;
            // ---- insert: unimodular row operations on b_j..b_h until the
            // coefficient vector is a unit vector at some position p, whose
            // row is then the new vector; move it to position j ----
            int p = 0;
            for (int guard = 0; guard < 4096; ++guard) {
                int cntnz = 0, pm = -1;
                if (z.lane == 0) {
                    for (int s = 0; s < n; ++s)
                        if (x[s]) {
                            ++cntnz;
                            if (pm < 0 || abs(x[s]) < abs(x[pm])) pm = s;
                        }
                    xc[0] = cntnz;
                    xc[1] = pm;
                }
                __syncthreads();
                cntnz = xc[0];
                pm = xc[1];
                __syncthreads();
                if (cntnz <= 1) {
                    p = pm;
                    break;
                }
                for (int s = 0; s < n; ++s) {
                    if (s == pm) continue;
                    const int xs = x[s];
                    if (!xs) continue;
                    const int xp = x[pm];
                    // floor division keeps the remainder in [0, |xp|)
                    int q = xs / xp;
                    if ((xs % xp != 0) && ((xs < 0) != (xp < 0))) --q;
                    __syncthreads();
                    if (z.lane == 0) x[s] = xs - q * xp;
                    // b_pm += q b_s keeps v = sum x b unchanged
                    for (int c = z.lane; c < dim; c += kW)
                        z.B[(size_t)(j + pm) * dim + c] += (int64_t)q * z.B[(size_t)(j + s) * dim + c];
                    __syncthreads();
                }
            }
            if (z.lane == 0 && x[p] < 0) x[p] = -x[p], xc[2] = 1;
            else if (z.lane == 0) xc[2] = 0;
            __syncthreads();
            const int neg = xc[2];
            // the new vector is row j+p (negated if its coefficient was -1);
            // rotate it to position j
            for (int c = z.lane; c < dim; c += kW) {
                const int64_t v = neg ? -z.B[(size_t)(j + p) * dim + c] : z.B[(size_t)(j + p) * dim + c];
                for (int s = p; s > 0; --s) z.B[(size_t)(j + s) * dim + c] = z.B[(size_t)(j + s - 1) * dim + c];
                z.B[(size_t)j * dim + c] = v;
            }
            __syncthreads();
            z.gram_all();
            z.lll(j, a.delta, budget);
            ++inserted;
            changed = 1;
        }
        if (!changed) break;
    }
    if (a.b_in_lds) {
        for (int e = z.lane; e < k * dim; e += kW) Bg[e] = Bs[e];
        __syncthreads();
    }
    if (z.lane == 0) {
        a.out[2 * inst] = z.flag[0] ? -4 : (budget > 0 ? 0 : -10);
        a.out[2 * inst + 1] = (int)inserted;
        a.nodes[inst] = nodes_total;
    }
}

size_t bkz_lds_bytes(int k) {
    return sizeof(long long) * (size_t)(k * (k + 1) / 2) + sizeof(double) * (size_t)(k * (k - 1) / 2 + 1 + 2 * k) +
           sizeof(int) * (size_t)(2 * k + 2) + sizeof(double) * (size_t)(2 * k + 1) + sizeof(int) * (size_t)(2 * k + 2) +
           64;
}

hipError_t launch_bkz(BkzArgs a, hipStream_t st) {
    size_t lds = bkz_lds_bytes(a.k);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const size_t with_b = lds + sizeof(int64_t) * (size_t)a.k * a.dim;
    a.b_in_lds = with_b <= 160 * 1024 ? 1 : 0;
    if (a.b_in_lds) lds = with_b;
    hipError_t e = hipFuncSetAttribute((const void *)bkz_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    if (a.count < 1 || (a.count > 1 && a.bstride < (int64_t)a.k * a.dim)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bkz_kernel, dim3(a.count), dim3(kW), lds, st, a);
    return hipGetLastError();
}

}  // namespace msp
