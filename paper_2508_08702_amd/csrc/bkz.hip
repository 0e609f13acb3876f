// Block Korkine-Zolotarev reduction of the kernel basis (paper, Section 2:
// the reduction step may use BKZ instead of LLL).  A better reduced basis
// leaves the solution set unchanged and shrinks the enumeration tree.
//
// One 64-lane wave per instance works on the k x dim int64 kernel basis in
// place.  The exact int64 Gram matrix (lower triangle) and the FP64
// Gram-Schmidt data (mu, beta) live in LDS.  The Gram matrix is computed from
// the basis once; every row operation (b_i += q b_j, an exchange, a sign
// change) then updates it exactly in O(k), and Gram-Schmidt rows are
// recomputed from it whenever the LLL loop visits a row.  A tour visits every
// block [j, h], h = min(j + beta, k) - 1:
//   * the wave finds a shortest nonzero vector of the block's projected
//     lattice by Schnorr-Euchner enumeration, one level per lane (radius
//     0.999 beta_j, shrunk to each shorter vector found, node cap per block);
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

// Broadcast of lane src's double to the whole wave (src uniform).
__device__ __forceinline__ double bcast(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, src);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Entries of the Gram diagonal stay <= 2^52, so every basis entry is at most
// 2^26 in absolute value and every Gram entry at most 2^52.  An update that
// would leave these bounds sets the overflow flag, and the caller keeps the
// LLL basis.
constexpr long long kGramMax = 1ll << 52;

struct Bkz {
    int k, dim;
    int64_t *B;        // k x dim (LDS or global)
    long long *G;      // Gram, lower triangle (LDS)
    double *mu;        // mu_{ij}, i > j (LDS)
    double *bb;        // beta_i = ||b*_i||^2 (LDS)
    int *flag;         // [0] overflow (LDS)
    int lane;

    __device__ long long &gram(int i, int j) const { return i >= j ? G[tri(i, j)] : G[tri(j, i)]; }

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

    // Gram-Schmidt row i from the exact Gram row and the rows < i
    // (Cholesky order): r_l = G_il - sum_{j<l} mu_lj r_j, mu_il = r_l / beta_l,
    // beta_i = G_ii - sum_l mu_il r_l.  Lane owns l = lane and lane + 64; once
    // r_j is final it is broadcast and subtracted from every later r_l, so the
    // dependent chain is one fused multiply-add per column.  The mu_lj of
    // kAhead columns are loaded together, ahead of the chain; a lane with
    // nothing to subtract uses a zero coefficient, which leaves its r_l as it is.
    static constexpr int kAhead = 8;
    template <bool HI, bool SRC1>
    __device__ void gs_cols(int i, int jb, int je, double &r0, double &r1) {
        const int l0 = lane, l1 = lane + kW;
        for (int j0 = jb; j0 < je; j0 += kAhead) {
            double c0[kAhead], c1[kAhead];
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                const int j = j0 + u;
                if (!SRC1) {
                    const bool v = l0 > j && l0 < i;
                    c0[u] = mu[v ? trs(l0, j) : 0];
                    if (!v) c0[u] = 0.0;
                }
                if (HI) {
                    const bool v = l1 > j && l1 < i;
                    c1[u] = mu[v ? trs(l1, j) : 0];
                    if (!v) c1[u] = 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < kAhead; ++u) {
                const int j = j0 + u;
                if (j < je) {
                    const double rj = SRC1 ? bcast(r1, j - kW) : bcast(r0, j);
                    if (!SRC1) r0 = fma(-c0[u], rj, r0);
                    if (HI) r1 = fma(-c1[u], rj, r1);
                }
            }
        }
    }

    __device__ void gs_row(int i) {
        const int l0 = lane, l1 = lane + kW;
        double r0 = l0 < i ? (double)gram(i, l0) : 0.0;
        double r1 = l1 < i ? (double)gram(i, l1) : 0.0;
        if (i > kW) {
            gs_cols<true, false>(i, 0, kW, r0, r1);
            gs_cols<true, true>(i, kW, i, r0, r1);
        } else {
            gs_cols<false, false>(i, 0, i, r0, r1);
        }
        double acc = 0.0;
        if (l0 < i) {
            const double m = r0 / bb[l0];
            mu[trs(i, l0)] = m;
            acc = m * r0;
        }
        if (l1 < i) {
            const double m = r1 / bb[l1];
            mu[trs(i, l1)] = m;
            acc += m * r1;
        }
        for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, kW);
        if (lane == 0) bb[i] = (double)gram(i, i) - acc;
        __syncthreads();
    }

    // b_i += q b_j in the basis and the Gram matrix (mu is left to the caller)
    __device__ void row_add(int i, int j, long long q) {
        for (int c = lane; c < dim; c += kW) B[(size_t)i * dim + c] += q * B[(size_t)j * dim + c];
        const long long gij = gram(i, j), gjj = gram(j, j), gii = gram(i, i);
        long long nl[2];
        bool bad = false;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int l = lane + h * kW;
            nl[h] = 0;
            if (l < k && l != i) {
                long long t;
                bad |= __builtin_mul_overflow(q, gram(j, l), &t);
                bad |= __builtin_add_overflow(gram(i, l), t, &nl[h]);
            }
        }
        // G_ii + 2 q G_ij + q^2 G_jj
        long long t1, t2, t3, nd;
        bad |= __builtin_mul_overflow(q, gij, &t1);
        bad |= __builtin_mul_overflow(t1, 2ll, &t1);
        bad |= __builtin_mul_overflow(q, gjj, &t2);
        bad |= __builtin_mul_overflow(t2, q, &t3);
        bad |= __builtin_add_overflow(gii, t1, &nd);
        bad |= __builtin_add_overflow(nd, t3, &nd);
        if (nd > kGramMax) bad = true;
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int l = lane + h * kW;
            if (l < k && l != i) gram(i, l) = nl[h];
        }
        if (lane == 0) gram(i, i) = nd;
        if (__ballot(bad) && lane == 0) flag[0] = 1;
        __syncthreads();
    }

    // exchange rows i and j of the basis and of the Gram matrix
    __device__ void swap_rows(int i, int j) {
        for (int c = lane; c < dim; c += kW) {
            const int64_t t = B[(size_t)i * dim + c];
            B[(size_t)i * dim + c] = B[(size_t)j * dim + c];
            B[(size_t)j * dim + c] = t;
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int l = lane + h * kW;
            if (l < k && l != i && l != j) {
                const long long t = gram(i, l);
                gram(i, l) = gram(j, l);
                gram(j, l) = t;
            }
        }
        if (lane == 0) {
            const long long t = gram(i, i);
            gram(i, i) = gram(j, j);
            gram(j, j) = t;
        }
        __syncthreads();
    }

    // b_i := -b_i
    __device__ void negate_row(int i) {
        for (int c = lane; c < dim; c += kW) B[(size_t)i * dim + c] = -B[(size_t)i * dim + c];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int l = lane + h * kW;
            if (l < k && l != i) gram(i, l) = -gram(i, l);
        }
        __syncthreads();
    }

    // Size reduction of row i against rows i-1, ..., 0 (|mu_ij| <= 0.51
    // afterwards).  The mu row is held in registers and reduced column by
    // column, the next column being the highest one over the threshold
    // (found by ballot); the multiples q_j are collected, and the basis row
    // and the Gram row are then updated once, b_i' = b_i - sum_j q_j b_j, with
    //   G_il' = G_il - sum_j q_j G_jl  (l != i),
    //   G_ii' = G_ii - sum_j q_j (G_ij + G_ij').
    // beta_i does not change.
    __device__ void size_reduce(int i) {
        const int l0 = lane, l1 = lane + kW;
        double m0 = l0 < i ? mu[trs(i, l0)] : 0.0;
        double m1 = l1 < i ? mu[trs(i, l1)] : 0.0;
        long long q0 = 0, q1 = 0;  // the multiples of rows l0 and l1
        int top = i;               // columns < top remain to be checked
        bool bad = false;
        for (;;) {
            const unsigned long long b1 = __ballot(l1 < top && fabs(m1) > 0.51);
            const unsigned long long b0 = __ballot(l0 < top && fabs(m0) > 0.51);
            int j;
            double mj;
            if (b1) {
                j = kW + 63 - __clzll(b1);
                mj = bcast(m1, j - kW);
            } else if (b0) {
                j = 63 - __clzll(b0);
                mj = bcast(m0, j);
            } else {
                break;
            }
            if (!(fabs(mj) < 1e9)) {  // no sensible integer multiple
                bad = true;
                break;
            }
            const long long q = (long long)rint(mj);
            if (l0 < j) m0 -= (double)q * mu[trs(j, l0)];
            if (l1 < j) m1 -= (double)q * mu[trs(j, l1)];
            if (l0 == j) m0 -= (double)q, q0 = q;
            if (l1 == j) m1 -= (double)q, q1 = q;
            top = j;
        }
        if (bad) {
            if (lane == 0) flag[0] = 1;
            __syncthreads();
            return;
        }
        if (top == i) return;
        // The new row's squared length, from the Gram-Schmidt data: beta_i +
        // sum_l mu_il'^2 beta_l.  While it is below 2^54, the exact values
        // below (a Gram row entry is at most the geometric mean of two
        // diagonal entries) all fit in int64, so wrapping int64 arithmetic
        // computes them exactly; the exact diagonal entry is then checked
        // against the estimate and against 2^52.
        double est = 0.0;
        if (l0 < i) est = m0 * m0 * bb[l0];
        if (l1 < i) est += m1 * m1 * bb[l1];
        for (int o = 32; o >= 1; o >>= 1) est += __shfl_xor(est, o, kW);
        est += bb[i];
        if (!(est < 0x1p54)) {
            if (lane == 0) flag[0] = 1;
            __syncthreads();
            return;
        }
        uint64_t bi[2], gold[2], gnew[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = lane + h * kW;
            bi[h] = c < dim ? (uint64_t)B[(size_t)i * dim + c] : 0;
            gold[h] = (c < k && c != i) ? (uint64_t)gram(i, c) : 0;
            gnew[h] = gold[h];
        }
        for (int h = 0; h < 2; ++h) {
            unsigned long long nz = __ballot((h ? q1 : q0) != 0);
            while (nz) {
                const int bit = __ffsll(nz) - 1;
                nz &= nz - 1;
                const int j = bit + h * kW;
                const long long qv = h ? q1 : q0;
                const uint64_t q = ((uint64_t)(unsigned)__builtin_amdgcn_readlane((int)(qv >> 32), bit) << 32) |
                                   (unsigned)__builtin_amdgcn_readlane((int)qv, bit);
#pragma unroll
                for (int g = 0; g < 2; ++g) {
                    const int c = lane + g * kW;
                    const uint64_t bj = (uint64_t)B[(size_t)j * dim + (c < dim ? c : 0)];
                    const uint64_t gj = (uint64_t)gram(j, c < k ? c : 0);
                    if (c < dim) bi[g] -= q * bj;
                    if (c < k && c != i) gnew[g] -= q * gj;
                }
            }
        }
        // G_ii' = G_ii - sum_j q_j (G_ij + G_ij')
        uint64_t d = 0;
        if (q0) d += (uint64_t)q0 * (gold[0] + gnew[0]);
        if (q1) d += (uint64_t)q1 * (gold[1] + gnew[1]);
        for (int o = 32; o >= 1; o >>= 1) d += (uint64_t)__shfl_xor((long long)d, o, kW);
        const long long nd = (long long)((uint64_t)gram(i, i) - d);
        if (nd > kGramMax || nd <= 0 || fabs((double)nd - est) > 0.5 * est + 1024.0) bad = true;
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int c = lane + h * kW;
            if (c < dim) B[(size_t)i * dim + c] = (int64_t)bi[h];
            if (c < k && c != i) gram(i, c) = (long long)gnew[h];
            if (c < i) mu[trs(i, c)] = h ? m1 : m0;
        }
        if (lane == 0) gram(i, i) = nd;
        if (__ballot(bad) && lane == 0) flag[0] = 1;
        __syncthreads();
    }

    // LLL (Lovasz delta) assuming rows < start have valid GS data
    __device__ void lll(int start, double delta, long long &budget) {
        int i = start < 1 ? 1 : start;
        if (start <= 0) gs_row(0);
        while (i < k && budget > 0 && !flag[0]) {
            --budget;
            gs_row(i);
            size_reduce(i);
            const double m1 = mu[trs(i, i - 1)];
            if (bb[i] >= (delta - m1 * m1) * bb[i - 1]) {
                ++i;
            } else {
                swap_rows(i - 1, i);
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
    int *x = reinterpret_cast<int *>(z.bb + k);  // block coefficients of the shortest vector found
    int *xc = x + k;                             // words lane 0 hands to the wave during an insertion
    z.flag = xc + 4;                             // [0] overflow
    if (z.lane == 0) z.flag[0] = 0;
    // the basis itself in LDS when it fits (copied back at the end)
    int64_t *Bs = reinterpret_cast<int64_t *>(smem + bkz_lds_bytes(k));
    if (a.b_in_lds) {
        for (int e = z.lane; e < k * dim; e += kW) Bs[e] = Bg[e];
        z.B = Bs;
    }
    __syncthreads();
    long long budget = a.max_lll_iters;
    z.gram_all();
    for (int i = z.lane; i < k; i += kW)
        if (z.gram(i, i) > kGramMax) z.flag[0] = 1;
    __syncthreads();
    z.lll(0, a.delta, budget);
    long long inserted = 0, nodes_total = 0;
    for (int tour = 0; tour < a.tours && !z.flag[0] && budget > 0; ++tour) {
        int changed = 0;
        for (int j = 0; j + 1 < k && !z.flag[0] && budget > 0; ++j) {
            const int h = (j + a.beta < k ? j + a.beta : k) - 1;
            const int n = h - j + 1;
            // ---- block SVP across the wave ----
            // Schnorr-Euchner enumeration of the projected block lattice:
            // level t (0 = block start j) takes values in zig-zag order
            // around its centre, so the first value beyond the radius ends the
            // level; while every coefficient above is zero only 0, 1, 2, ...
            // are taken (v and -v are the same vector).  Lane t holds level
            // t: its value X, centre C, the partial norm Lp of the levels
            // above, and the zig-zag start.  Centres are kept current: a
            // change of x_s by D moves every lower centre by -D mu_{s,t}, one
            // fused multiply-add per lane, with the mu rows the step may need
            // loaded at the top of each node.
            int found = 0;
            {
                const int lane = z.lane;
                const double bt = lane < n ? z.bb[j + lane] : 0.0;
                int X = 0, U1 = 0, S = 1, TZ = 0, BX = 0;
                double C = 0.0, Lp = 0.0;
                if (lane == n - 1) TZ = 1;  // the top level starts at 0, one direction
                double R = z.bb[j] * 0.999;
                long long nodes = 0;
                int t = n - 1;
                while (nodes < a.max_nodes) {
                    ++nodes;
                    const bool vm = t >= 1 && lane < t - 1, v0 = lane < t, vp = t + 1 < n && lane < t + 1;
                    double mrm = z.mu[vm ? trs(j + t - 1, j + lane) : 0];
                    double mr0 = z.mu[v0 ? trs(j + t, j + lane) : 0];
                    double mrp = z.mu[vp ? trs(j + t + 1, j + lane) : 0];
                    if (!vm) mrm = 0.0;
                    if (!v0) mr0 = 0.0;
                    if (!vp) mrp = 0.0;
                    const int xt = __builtin_amdgcn_readlane(X, t);
                    const double dx = (double)xt - bcast(C, t);
                    const double l = dx * dx * bcast(bt, t) + bcast(Lp, t);
                    int tn = t;  // the level whose value advances
                    double mrow = mr0;
                    if (l < R) {
                        if (t > 0) {
                            // down one level: start it at the value nearest its centre
                            const int tz = __builtin_amdgcn_readlane(TZ, t) && xt == 0;
                            const double c = bcast(C, t - 1);
                            const int u1 = tz ? 0 : (int)rint(c);
                            const int s0 = ((double)u1 - c <= 0.0) ? 1 : -1;
                            if (lane == t - 1) {
                                Lp = l;
                                TZ = tz;
                                U1 = u1;
                                S = s0;
                                X = u1;
                            }
                            C = fma(-(double)u1, mrm, C);
                            --t;
                            continue;
                        }
                        if (__ballot(X != 0)) {  // a nonzero vector shorter than the radius
                            R = l;
                            BX = X;
                            found = 1;
                        }
                    } else {
                        // level t is exhausted: its value returns to 0, up one level
                        C = fma((double)xt, mr0, C);
                        if (lane == t) X = 0;
                        ++t;
                        if (t >= n) break;
                        tn = t;
                        mrow = mrp;
                    }
                    // next value of level tn
                    const int x0 = __builtin_amdgcn_readlane(X, tn);
                    int nx;
                    if (__builtin_amdgcn_readlane(TZ, tn)) {
                        nx = x0 + 1;
                    } else {
                        const int u1 = __builtin_amdgcn_readlane(U1, tn);
                        const int s0 = __builtin_amdgcn_readlane(S, tn);
                        const int off = x0 - u1;
                        int no;
                        if (off == 0)
                            no = s0;
                        else if ((off > 0) == (s0 > 0))
                            no = -off;
                        else
                            no = -off + s0;
                        nx = u1 + no;
                    }
                    if (lane == tn) X = nx;
                    C = fma(-(double)(nx - x0), mrow, C);
                }
                nodes_total += nodes;
                if (found && lane < n) x[lane] = BX;
                __syncthreads();
            }
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
                    z.row_add(j + pm, j + s, q);
                }
            }
            if (z.lane == 0 && x[p] < 0) x[p] = -x[p], xc[2] = 1;
            else if (z.lane == 0) xc[2] = 0;
            __syncthreads();
            const int neg = xc[2];
            // the new vector is row j+p (negated if its coefficient was -1);
            // move it to position j by adjacent exchanges
            if (neg) z.negate_row(j + p);
            for (int s = p; s > 0; --s) z.swap_rows(j + s - 1, j + s);
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

// LDS of one workgroup without the basis: the Gram triangle, mu (and one
// spare), beta, the block coefficients, the broadcast words and the flag,
// rounded up to 8 bytes (the basis follows when it fits).
__host__ __device__ size_t bkz_lds_bytes(int k) {
    const size_t b = sizeof(long long) * (size_t)(k * (k + 1) / 2) + sizeof(double) * (size_t)(k * (k - 1) / 2 + 1 + k) +
                     sizeof(int) * (size_t)(k + 4 + 2);
    return (b + 7) & ~(size_t)7;
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
