// Subtree root generation: the top levels of the enumeration tree, expanded
// breadth first (tree partitioning, paper Section 4): a level of more than
// kThinMax parents per count launch, scan and write launch; runs of smaller
// levels in one single-workgroup launch (expand_thin_kernel).
//
// A level-t launch takes the expanded nodes of level t+1 ("parents", each with
// its prefix u_{t+1..k-1}, projected vector w^(t+1) and partial norm) and, one
// thread per parent, runs the level-t rules of Algorithm 1: zig-zag values
// around the centre, the l2 bound, the Hoelder test and the one-direction
// cut.  Every candidate that passes both tests is an expanded node of level t.
// A count pass, an exclusive scan (rocPRIM) and a write pass store the children of
// parent p contiguously after those of parent p-1, each parent's children in
// zig-zag order -- so every level of the frontier is in depth-first order, and
// the last frontier is the root queue in the order sequential DFS meets it.
#include <rocprim/device/device_scan.hpp>

#include "enum_rules.h"
#include "expand_thin.h"
#include "msp_internal.h"

namespace msp {

namespace {

// A thread works alone on its parent, so every loop below issues the loads of
// kChunk elements before it uses any of them: one memory round trip per chunk
// instead of one per element.  The loads are unconditional (an index past the
// end is clamped to the last element, whose value is then not used), so the
// compiler needs no branch, and no wait, per element.  Each sum keeps its
// element order, so results are bit-identical to the plain loops.
constexpr int kChunk = 16;

// centre_natural's sum (term p = k-1-i into partial sum p mod 4, fused
// multiply-adds in increasing p), with batched loads
__device__ __forceinline__ double centre_batched(const int8_t *__restrict__ u, const double *__restrict__ mu, int k,
                                                 int t) {
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    const int nt = k - 1 - t;
    for (int p0 = 0; p0 < nt; p0 += kChunk) {
        double uv[kChunk], mv[kChunk];
#pragma unroll
        for (int r = 0; r < kChunk; ++r) {
            const int p = p0 + r < nt ? p0 + r : nt - 1, i = k - 1 - p;
            uv[r] = (double)u[i];
            mv[r] = mu[(size_t)i * k + t];
        }
#pragma unroll
        for (int r = 0; r < kChunk; ++r)
            if (p0 + r < nt) s[r & 3] = fma(uv[r], mv[r], s[r & 3]);
    }
    return combine4(s[0], s[1], s[2], s[3]);
}

// sum_j |x b_t[j] + w[j]| over j = 0 .. dim-1 in increasing j
__device__ __forceinline__ double l1_batched(double x, const double *__restrict__ bt, const double *__restrict__ wp,
                                             int64_t pw, int dim) {
    double h = 0.0;
    for (int j0 = 0; j0 < dim; j0 += kChunk) {
        double pv[kChunk], bv[kChunk];
#pragma unroll
        for (int r = 0; r < kChunk; ++r) {
            const int j = j0 + r < dim ? j0 + r : dim - 1;
            pv[r] = wp[(size_t)j * pw];
            bv[r] = bt[j];
        }
#pragma unroll
        for (int r = 0; r < kChunk; ++r)
            if (j0 + r < dim) h += fabs(fma(x, bv[r], pv[r]));
    }
    return h;
}

// The level-t rules for parent p: returns its number of children and adds
// its evaluations, nodes and expansions to ce, cn, cx.  WRITE: the children
// are stored from slot on.
template <bool WRITE>
__device__ __forceinline__ int64_t expand_parent(const ExpandArgs &a, int64_t p, int64_t slot,
                                                 unsigned long long &ce, unsigned long long &cn,
                                                 unsigned long long &cx) {
    {
        const int k = a.k, dim = a.dim, t = a.t;
        const int8_t *__restrict__ up = a.par.u + p * k;
        const double *__restrict__ wp = a.par.w + p;  // column-major: element j at wp[j * pw]
        const int64_t pw = a.par.wcap;
        const double lpar = a.par.l[p];
        const bool tz = a.par.tz[p] != 0;
        const int pd = a.par.dsc[p];
        const double y = centre_batched(up, a.mu, k, t);
        const Zig z = zig_init(y, tz);
        int u = z.u1;
        bool onedir = tz;
        int dir = 1;
        const double beta = a.beta[t];
        const double *__restrict__ bt = a.bhat + (size_t)t * dim;
        int64_t nch = 0;
        for (;;) {
            // a budget stops the level at the first value whose cost would
            // take the path beyond it
            const int rank = disc_cost(z, u, tz, a.disc_count != 0);
            if (a.budget >= 0 && pd + rank > a.budget) break;
            const double x = add_rn((double)u, y);
            const double l = partial_norm(x, beta, lpar);
            ++ce;
            if (!(l <= a.bound)) break;  // NaN ends the level too
            ++cn;
            bool fail = false;
            if (a.hoelder) {
                const double h = l1_batched(x, bt, wp, pw, dim);
                fail = l > (a.rmax * h) * a.hfac;
            }
            if (fail) {
                if (a.onedir) {
                    if (onedir) break;
                    u = zig_next(z, u);
                    onedir = true;
                    dir = side_of(u, y);
                    continue;
                }
            } else {
                ++cx;
                if (WRITE) {
                    if (u > 127 || u < -127) atomicOr(&a.flags[1], 1);
                    int8_t *__restrict__ uc = a.ch.u + slot * k;
                    for (int i0 = 0; i0 < k; i0 += kChunk) {
                        int8_t v[kChunk];
#pragma unroll
                        for (int r = 0; r < kChunk; ++r) {
                            v[r] = up[i0 + r < k ? i0 + r : k - 1];
                        }
#pragma unroll
                        for (int r = 0; r < kChunk; ++r) {
                            const int i = i0 + r;
                            if (i < k) uc[i] = i > t ? v[r] : (i == t ? (int8_t)u : (int8_t)0);
                        }
                    }
                    double *__restrict__ wc = a.ch.w + slot;
                    const int64_t cw = a.ch.wcap;
                    for (int j0 = 0; j0 < a.dimp; j0 += kChunk) {
                        double pv[kChunk], bv[kChunk];
#pragma unroll
                        for (int r = 0; r < kChunk; ++r) {
                            const int j = j0 + r < dim ? j0 + r : dim - 1;
                            pv[r] = wp[(size_t)j * pw];
                            bv[r] = bt[j];
                        }
#pragma unroll
                        for (int r = 0; r < kChunk; ++r) {
                            const int j = j0 + r;
                            if (j < a.dimp) wc[(size_t)j * cw] = j < dim ? fma(x, bv[r], pv[r]) : 0.0;
                        }
                    }
                    a.ch.l[slot] = l;
                    a.ch.tz[slot] = (tz && u == 0) ? 1 : 0;
                    a.ch.dsc[slot] = (uint8_t)(pd + rank < 255 ? pd + rank : 255);
                    ++slot;
                }
                ++nch;
            }
            u = onedir ? u + dir : zig_next(z, u);
        }
        return nch;
    }
}

// Wave sums of the counters, one atomic add each per wave.
__device__ __forceinline__ void add_counters(unsigned long long *counters, unsigned long long ce,
                                             unsigned long long cn, unsigned long long cx) {
    for (int o = 32; o >= 1; o >>= 1) {
        ce += __shfl_xor(ce, o, 64);
        cn += __shfl_xor(cn, o, 64);
        cx += __shfl_xor(cx, o, 64);
    }
    if ((threadIdx.x & 63) == 0 && (ce | cn | cx)) {
        atomicAdd(&counters[0], ce);
        atomicAdd(&counters[1], cn);
        atomicAdd(&counters[2], cx);
    }
}

}  // namespace

template <bool WRITE>
__global__ void __launch_bounds__(256) expand_kernel(ExpandArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long ce = 0, cn = 0, cx = 0;
    if (p < a.np) {
        const int64_t nch = expand_parent<WRITE>(a, p, WRITE ? a.offs[p] : 0, ce, cn, cx);
        if (!WRITE) a.counts[p] = nch;
    }
    if (WRITE) add_counters(a.counters, ce, cn, cx);
}

// Thin levels in one launch: one workgroup expands level after level while
// the parents number at most kThinMax, with the count pass, an exclusive scan
// of the counts in LDS and the write pass of each level separated by
// barriers.  It takes the same levels as the per-level launches would (the
// same stop rule, the same capacity check, children in the same slots), so
// the frontier and the counters are identical; what it saves is the host
// round trip and the four launches of every level.  The frontier it ends on
// is in fr[out->cur].
__global__ void __launch_bounds__(kThinBlock) expand_thin_kernel(ThinArgs a) {
    __shared__ int cnt[kThinMax];
    __shared__ int64_t off[kThinMax];
    __shared__ int64_t wsum[kThinBlock / 64];
    __shared__ int64_t total_s;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int64_t np = a.np;
    int L = a.L, cur = 0, capped = 0;
    unsigned long long ce = 0, cn = 0, cx = 0;
    while (L - 1 >= 1 && np <= kThinMax && !thin_done(a.rule, np, L)) {
        ExpandArgs e = a.e;
        e.t = L - 1;
        e.par = a.fr[cur];
        e.ch = a.fr[cur ^ 1];
        e.np = np;
        unsigned long long de = 0, dn = 0, dx = 0;  // the count pass adds no counters
        for (int64_t p = tid; p < np; p += kThinBlock) cnt[p] = (int)expand_parent<false>(e, p, 0, de, dn, dx);
        __syncthreads();
        // exclusive scan: thread tid owns cnt[tid * kThinPer ..] (kThinPer entries)
        int64_t own = 0;
        for (int i = 0; i < kThinPer; ++i) {
            const int64_t q = (int64_t)tid * kThinPer + i;
            if (q < np) own += cnt[q];
        }
        int64_t x = own;  // inclusive sum over the wave
        for (int o = 1; o < 64; o <<= 1) {
            const int64_t y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wsum[wave] = x;
        __syncthreads();
        if (tid == 0) {
            int64_t acc = 0;
            for (int w = 0; w < kThinBlock / 64; ++w) {
                const int64_t v = wsum[w];
                wsum[w] = acc;
                acc += v;
            }
            total_s = acc;
        }
        __syncthreads();
        int64_t base = wsum[wave] + x - own;
        for (int i = 0; i < kThinPer; ++i) {
            const int64_t q = (int64_t)tid * kThinPer + i;
            if (q < np) {
                off[q] = base;
                base += cnt[q];
            }
        }
        const int64_t total = total_s;
        __syncthreads();
        if (total > a.fcap) {  // this level would not fit the frontier buffers
            capped = 1;
            break;
        }
        for (int64_t p = tid; p < np; p += kThinBlock) expand_parent<true>(e, p, off[p], ce, cn, cx);
        __syncthreads();  // the children are the next level's parents
        cur ^= 1;
        np = total;
        L = e.t;
        if (np == 0) break;
    }
    add_counters(a.e.counters, ce, cn, cx);
    if (tid == 0) {
        a.out->np = np;
        a.out->L = L;
        a.out->cur = cur;
        a.out->capped = capped;
    }
}

__global__ void frontier_init_kernel(Frontier f, int k, int ws) {
    for (int i = threadIdx.x; i < k; i += blockDim.x) f.u[i] = 0;
    for (int j = threadIdx.x; j < ws; j += blockDim.x) f.w[(size_t)j * f.wcap] = 0.0;
    if (threadIdx.x == 0) {
        f.l[0] = 0.0;
        f.tz[0] = 1;
        f.dsc[0] = 0;
    }
}

// total = offs[n-1] + counts[n-1] after the exclusive scan
__global__ void scan_total_kernel(const int64_t *counts, const int64_t *offs, int64_t n, int64_t *total) {
    if (threadIdx.x == 0) *total = n > 0 ? offs[n - 1] + counts[n - 1] : 0;
}

// Root generation's last frontier becomes the first pool items: level L-1,
// prefix u_{L..k-1}, starting at the level's first value.
__global__ void pool_init_kernel(Frontier f, int64_t nroots, int k, int L, Pool pool) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nroots) {
        for (int j = 0; j < k; ++j) pool.u[i * k + j] = j >= L ? f.u[i * k + j] : (int8_t)0;
        pool.meta[i] = make_int4(L - 1, 0, 8 | (f.tz[i] ? 4 : 0), f.dsc[i]);
        pool.ready[i] = 1;
    }
    for (int64_t j = nroots + i; j < pool.cap; j += (int64_t)gridDim.x * blockDim.x) pool.ready[j] = 0;
}

// Copy frontier records idx[0..n) of src into dst[0..n) (one wave per record).
__global__ void gather_frontier_kernel(Frontier src, const int64_t *idx, int64_t base, int64_t n, Frontier dst, int k,
                                       int ws) {
    const int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x & 63;
    if (r >= n) return;
    const int64_t s = idx ? idx[r] : base + r;
    for (int j = lane; j < ws; j += 64) dst.w[(size_t)j * dst.wcap + r] = src.w[(size_t)j * src.wcap + s];
    for (int j = lane; j < k; j += 64) dst.u[r * k + j] = src.u[s * k + j];
    if (lane == 0) {
        dst.l[r] = src.l[s];
        dst.tz[r] = src.tz[s];
        dst.dsc[r] = src.dsc[s];
    }
}

// Work items "enumerate level L-1 below the prefix" for records idx[0..n) of
// a frontier at level L (the walker recomputes w and the norms from u).
__global__ void frontier_items_kernel(Frontier src, const int64_t *idx, int64_t n, int k, int L, int8_t *iu,
                                      int4 *imeta) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t s = idx[r];
    for (int j = 0; j < k; ++j) iu[r * k + j] = j >= L ? src.u[s * k + j] : (int8_t)0;
    imeta[r] = make_int4(L - 1, 0, 8 | (src.tz[s] ? 4 : 0), src.dsc[s]);
}

__global__ void fill_int_kernel(int *p, int64_t n, int v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

static inline unsigned grid_for(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_gather_frontier(Frontier src, const int64_t *idx, int64_t base, int64_t n, Frontier dst, int k,
                                  int ws, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_frontier_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, src, idx, base, n, dst,
                       k, ws);
    return hipGetLastError();
}

hipError_t launch_frontier_items(Frontier src, const int64_t *idx, int64_t n, int k, int L, int8_t *iu, int4 *imeta,
                                 hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(frontier_items_kernel, dim3(grid_for(n)), dim3(256), 0, st, src, idx, n, k, L, iu, imeta);
    return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int64_t n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill_int_kernel, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_expand_count(const ExpandArgs &a, hipStream_t st) {
    if (a.np <= 0) return hipSuccess;
    hipLaunchKernelGGL(expand_kernel<false>, dim3(grid_for(a.np)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_expand_write(const ExpandArgs &a, hipStream_t st) {
    if (a.np <= 0) return hipSuccess;
    hipLaunchKernelGGL(expand_kernel<true>, dim3(grid_for(a.np)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_expand_thin(const ThinArgs &a, hipStream_t st) {
    if (a.np <= 0 || a.np > kThinMax) return hipErrorInvalidValue;
    hipLaunchKernelGGL(expand_thin_kernel, dim3(1), dim3(kThinBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_frontier_init(Frontier f, int k, int ws, hipStream_t st) {
    hipLaunchKernelGGL(frontier_init_kernel, dim3(1), dim3(256), 0, st, f, k, ws);
    return hipGetLastError();
}

hipError_t launch_pool_init(Frontier f, int64_t nroots, int k, int L, Pool pool, hipStream_t st) {
    const int64_t n = nroots > (1 << 18) ? nroots : (1 << 18);
    hipLaunchKernelGGL(pool_init_kernel, dim3(grid_for(n)), dim3(256), 0, st, f, nroots, k, L, pool);
    return hipGetLastError();
}

hipError_t launch_scan(void *temp, size_t *temp_bytes, const int64_t *counts, int64_t *offs, int64_t n,
                       int64_t *total, hipStream_t st) {
    if (!temp)
        return rocprim::exclusive_scan(nullptr, *temp_bytes, counts, offs, (int64_t)0, (size_t)n,
                                       rocprim::plus<int64_t>(), st);
    if (n > 0) {
        hipError_t e = rocprim::exclusive_scan(temp, *temp_bytes, counts, offs, (int64_t)0, (size_t)n,
                                               rocprim::plus<int64_t>(), st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(scan_total_kernel, dim3(1), dim3(64), 0, st, counts, offs, n, total);
    return hipGetLastError();
}

}  // namespace msp
