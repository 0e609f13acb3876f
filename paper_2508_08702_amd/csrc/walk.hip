// Persistent subtree walker: Algorithm 1 (paper, Section 2) below the split
// level, one work item per lane.
//
// Work items.  An item is (level T, prefix u_{T+1..k-1}, zig-zag
// continuation at level T): "enumerate the remaining values of u_T after the
// given prefix, and everything below them".  Root generation supplies the
// first items (T = split level - 1, continuation = the level's first value).
// Items sit in an HBM pool.  A lane without work takes a ticket (one atomic
// add on the head counter per wave, ranks by ballot prefix count); ticket i
// is pool slot i, and the lane waits until that slot holds an item.  While
// head > tail -- lanes are waiting -- every busy lane donates the untried
// values of its highest open level as a new item appended at the tail (tree
// partitioning, paper Section 4), so the work is split dynamically and no
// lane is left with a huge subtree at the end.  A count of unfinished items
// (pending) ends the walk: a waiting lane stops once it reaches zero.  A lane that takes an item
// recomputes centres, partial norms and w for the prefix, top level first, in
// the same order as the oracle; evaluations are never duplicated, so the
// search-tree counters are exactly those of a sequential run.
//
// Per-lane state.  w (Section 2: w^(t) = x_t b_hat_t + w^(t+1)) lives in DIMP
// registers and is updated incrementally: a new candidate at level t adds
// (u - u_applied) b_hat_t, or x b_hat_t on first use of the level, and
// leaving level t subtracts the applied x_t b_hat_t.  Each loop iteration
// performs exactly one such row update per lane, so all lanes run the
// expensive pass in lockstep; the cheap scalar control around it diverges.
// The state of the level above (centre, partial norm, beta, u, flags) is kept
// in registers, so popping a level waits for no memory; the level above that
// is fetched from the per-walker HBM stack while the walk goes on.
//
// LDS.  Rows b_hat_0..b_hat_{L-1} with a padded stride S (a multiple of 16
// doubles) and a wrap-around copy of the first 14 columns.  Lane l keeps w in
// the column order rotated by r = 2 (l mod 8): register j holds column
// (j + r) mod DIMP and the pass reads row[r + j], so eight lanes reading
// eight arbitrary rows hit eight distinct 16-byte bank groups.  Only l1
// norms and elementwise updates touch w; both ignore the column order.
// mu is stored by columns (column t = mu_{k-1,t}, mu_{k-2,t}, ..., mu_{t+1,t},
// zero padded to a multiple of 8) and each thread keeps its u values in a
// reversed int8 row, so a centre sum reads 8 levels per chunk.
#include "enum_rules.h"
#include "msp_internal.h"

namespace msp {

namespace {

enum : int { NEED_ROOT = 0, RUN = 1, DONE = 2, WAIT = 3, LOAD = 4 };
enum : int { K_NONE = 0, K_NODE = 1, K_REVERT = 2 };
enum : int { F_ONEDIR = 1, F_DIRPOS = 2, F_TZ = 4, F_FRESH = 8 };

constexpr int kRot = 2;  // rotation granule (columns): 128-bit reads
#ifndef MSP_WALK_INNER
#define MSP_WALK_INNER 1024
#endif
// Row layout in LDS.  The two-wave variant rotates each lane's columns by
// 2 (lane mod 16) and aligns every row to 1 KB, so 16 lanes reading 16
// arbitrary rows hit 16 distinct 16-byte bank groups; the one-wave variant
// rotates by 2 (lane mod 8) with 128-byte rows (a stored root's w carries
// padding for 8 rotations only).
__host__ __device__ constexpr int row_rots(bool two_wave) { return two_wave ? 16 : 8; }
__host__ __device__ constexpr int row_wrap(bool two_wave) { return 2 * (row_rots(two_wave) - 1); }
__host__ __device__ constexpr int row_align(bool two_wave) { return two_wave ? 128 : 16; }
__host__ __device__ constexpr int row_stride(int dimp, bool two_wave) {
    return ((dimp + row_wrap(two_wave) + row_align(two_wave) - 1) / row_align(two_wave)) * row_align(two_wave);
}

__device__ __forceinline__ unsigned long long wall_clock() { return wall_clock64(); }

// Flags are polled with relaxed loads.  An acquire load at agent scope also
// invalidates the wave's caches (the L2 of its XCD included), and the rare-work
// pass polls every few iterations, so the one flag whose data a lane then
// reads (a donated pool slot) is followed by a single acquire fence instead.
__device__ __forceinline__ int ld_rlx(const int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_rlx(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ long long ld_rlx(const long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Centre sum of level t in the fixed order (term p = k-1-i into partial sum
// p mod 4, fused multiply-adds; the order of centre_natural): one chunk of 8
// levels feeds each partial sum twice.  my_u[p] holds u_{k-1-p}; col[p] =
// mu_{k-1-p,t}, zero beyond the column's k-1-t entries (a zero term leaves a
// partial sum unchanged).  The loads of chunk c+1 are issued before chunk c
// is summed.
__device__ __forceinline__ double centre_sum(int t, int k, const int8_t *my_u, const double *col) {
    const int nt = k - 1 - t;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (nt <= 0) return 0.0;
    uint2 uu = *reinterpret_cast<const uint2 *>(my_u);
    double2 m0 = *reinterpret_cast<const double2 *>(col);
    double2 m1 = *reinterpret_cast<const double2 *>(col + 2);
    double2 m2 = *reinterpret_cast<const double2 *>(col + 4);
    double2 m3 = *reinterpret_cast<const double2 *>(col + 6);
    for (int c = 0; c < nt; c += 8) {
        const int cn = c + 8 < nt ? c + 8 : c;  // next chunk (re-read the current one at the end)
        const uint2 nu = *reinterpret_cast<const uint2 *>(my_u + cn);
        const double2 n0 = *reinterpret_cast<const double2 *>(col + cn);
        const double2 n1 = *reinterpret_cast<const double2 *>(col + cn + 2);
        const double2 n2 = *reinterpret_cast<const double2 *>(col + cn + 4);
        const double2 n3 = *reinterpret_cast<const double2 *>(col + cn + 6);
        s0 = fma((double)(int8_t)(uu.x), m0.x, s0);
        s1 = fma((double)(int8_t)(uu.x >> 8), m0.y, s1);
        s2 = fma((double)(int8_t)(uu.x >> 16), m1.x, s2);
        s3 = fma((double)(int8_t)(uu.x >> 24), m1.y, s3);
        s0 = fma((double)(int8_t)(uu.y), m2.x, s0);
        s1 = fma((double)(int8_t)(uu.y >> 8), m2.y, s1);
        s2 = fma((double)(int8_t)(uu.y >> 16), m3.x, s2);
        s3 = fma((double)(int8_t)(uu.y >> 24), m3.y, s3);
        uu = nu;
        m0 = n0;
        m1 = n1;
        m2 = n2;
        m3 = n3;
    }
    return combine4(s0, s1, s2, s3);
}

// A work item's prefix from the pool into the lane's LDS u row: my_u[k-1-j]
// = pu[j] for j > T, 0 below.  The global loads of 16 bytes are issued before
// any of them is stored (the index is clamped to the row, so every load is
// unconditional): one memory round trip per 16 bytes, not per byte.
__device__ __forceinline__ void load_prefix(int8_t *my_u, const int8_t *__restrict__ pu, int k, int T) {
    for (int j0 = 0; j0 < k; j0 += 16) {
        int8_t v[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) v[r] = pu[j0 + r < k ? j0 + r : k - 1];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int j = j0 + r;
            if (j < k) my_u[k - 1 - j] = j > T ? v[r] : (int8_t)0;
        }
    }
}

}  // namespace

__host__ __device__ int walk_row_stride(int dimp, int block) { return row_stride(dimp, block == 512); }
// per-thread u row: an odd number of 8-byte words, so 16 lanes reading the
// same word index hit 16 distinct bank pairs
__host__ __device__ int walk_u_stride(int k) {
    const int w8 = (k + 7) / 8;
    return 8 * (w8 | 1);
}
// mu column t starts 2 (t mod 8) doubles past a 16-double boundary, so lanes
// on levels with different t mod 8 read different 16-byte bank groups
__host__ __device__ int walk_muc_offset(int k, int t) {
    int off = 0;
    for (int tt = 0; tt <= t; ++tt) {
        off = ((off + 15) / 16) * 16 + 2 * (tt & 7);
        if (tt < t) off += ((k - 1 - tt + 7) / 8) * 8;
    }
    return off;
}

size_t walk_lds_bytes(int dimp, int block, int k, int L, int muc_len) {
    const int S = walk_row_stride(dimp, block);
    return sizeof(double) * ((size_t)L * S + (size_t)muc_len + (size_t)k) + sizeof(int) * (size_t)((k + 2) & ~1) +
           (size_t)walk_u_stride(k) * block;
}

// Layouts used by the walker: rotated rows (k x S) and mu by columns.
__global__ void walk_prep_kernel(int k, int dim, int dimp, int block, const double *bhat, const double *mu,
                                 double *g_bh, double *g_muc, int *g_coff) {
    const int S = walk_row_stride(dimp, block);
    const int wrap = row_wrap(block == 512);
    const int t = blockIdx.x;
    if (t < k) {
        for (int p = threadIdx.x; p < S; p += blockDim.x) {
            double v = 0.0;
            if (p < dimp + wrap) {
                const int c = p < dimp ? p : p - dimp;
                if (c < dim) v = bhat[(size_t)t * dim + c];
            }
            g_bh[(size_t)t * S + p] = v;
        }
        const int off = walk_muc_offset(k, t);
        const int nt = k - 1 - t, np = ((nt + 7) / 8) * 8;
        for (int p = threadIdx.x; p < np; p += blockDim.x)
            g_muc[off + p] = p < nt ? mu[(size_t)(k - 1 - p) * k + t] : 0.0;
        if (threadIdx.x == 0) {
            g_coff[t] = off;
            if (t == k - 1) g_coff[k] = off + np;
        }
    }
}

// BUDGETED: a discrepancy budget is set (a.budget >= 0); without one the
// discrepancy bookkeeping is compiled out.
//
// Register economy.  w takes DIMP registers; everything else a lane keeps
// between iterations is a handful of scalars (the level, its value and
// zig-zag state, one word of flags, the centre and partial norms of the
// level and its parent, 32-bit counters), so that at DIMP <= 88 two waves
// fit on a SIMD.  The parent level's state is cached in registers and the
// grandparent is read back from the per-walker stack on a pop.
//
// ALLROWS (the two-wave variant): every row b_hat_0..b_hat_{k-1} is in LDS,
// and a lane that takes an item rebuilds the prefix's w with ordinary row
// updates of the inner loop, one prefix level per iteration (state LOAD),
// which keeps the rare-work pass small.  Otherwise only rows below the split
// level are in LDS.  A root's w is then loaded as root generation stored it;
// an item donated below a root starts from that root's stored w and norm (the
// pool records which root an item descends from) and adds the levels below
// the roots' level in state LOAD as well; an item with no stored root above it
// (refinement leftovers) is rebuilt in the rare-work pass from the rows in HBM.
template <int DIMP, int BLOCK, bool BUDGETED>
__global__ void __launch_bounds__(BLOCK) walk_kernel(WalkArgs a) {
    constexpr bool ALLROWS = BLOCK == 512;
    constexpr int S = row_stride(DIMP, ALLROWS);
    constexpr int kInner = MSP_WALK_INNER;  // most iterations of the inner loop between rare-work passes
    extern __shared__ __align__(16) unsigned char smem[];
    const int k = a.k, L = ALLROWS ? a.k : a.L, tid = threadIdx.x;
    double *const stack_base = a.stack;
    int *const flagsp = a.flags;
    const int KU = walk_u_stride(k);
    double *s_bh = reinterpret_cast<double *>(smem);  // L x S
    double *s_muc = s_bh + (size_t)L * S;             // mu columns
    double *s_beta = s_muc + a.muc_len;               // k
    int *s_coff = reinterpret_cast<int *>(s_beta + k);  // k + 1 (padded to even)
    int8_t *s_u = reinterpret_cast<int8_t *>(s_coff + ((k + 2) & ~1));  // BLOCK x KU

    for (int idx = tid; idx < L * S; idx += BLOCK) s_bh[idx] = a.g_bh[idx];
    for (int idx = tid; idx < a.muc_len; idx += BLOCK) s_muc[idx] = a.g_muc[idx];
    for (int q = tid; q < k; q += BLOCK) s_beta[q] = a.beta[q];
    for (int q = tid; q <= k; q += BLOCK) s_coff[q] = a.g_coff[q];
    for (int idx = tid; idx < KU * BLOCK; idx += BLOCK) s_u[idx] = 0;
    __syncthreads();

    const int lane = tid & 63;
    const int rot = kRot * (lane & (row_rots(ALLROWS) - 1));  // this lane's column rotation
    int8_t *my_u = s_u + tid * KU;  // my_u[k-1-j] = u_j
    const double bound = a.bound, hfac = a.hfac, rmax_d = a.rmax_d;
    const bool hoelder = a.hoelder != 0, onedir_cut = a.onedir != 0;
    const int budget = a.budget;
    const bool dcount = a.disc_count != 0;
    // this walker's stack: k entries of {centre, partial norm of the parent,
    // flags, discrepancies}, level-major (level l of walker g at (l * walkers +
    // g) * 4).  The walker index is rebuilt from the wave's first index (one
    // scalar) and the lane id wherever it is needed, so no per-lane address
    // has to stay live across the inner loop.
    // (The lane id comes from v_mbcnt in a volatile block, which the compiler
    // can neither hoist nor keep live; entry indices fit in 32 bits: at most
    // 128 levels x 2^17 walkers.)
    const unsigned wave_first = __builtin_amdgcn_readfirstlane(blockIdx.x * BLOCK + (tid & ~63));
    const unsigned walkers = gridDim.x * BLOCK;
    auto stack_at = [&](int level) -> double * {
        unsigned ln;
        asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(ln));
        const unsigned e = (unsigned)level * walkers + wave_first + ln;
        return stack_base + (size_t)e * 4;
    };

    double w[DIMP];
#pragma unroll
    for (int j = 0; j < DIMP; ++j) w[j] = 0.0;

    int state = NEED_ROOT;
    int fex = 0, leafpend = 0, fin = 0;
    unsigned ticket = 0;
    int t = 0, u = 0, top = 0, u_app = 0;
    int onedir = 0, dir = 1, tz = 0, applied = 0;
    Zig z{0, 1};
    double y = 0.0, lpar = 0.0, lcur = 0.0, bt = 1.0;
    double Py = 0.0, Pl = 0.0;  // cached state of level t+1: centre and the partial norm above it
    int Pw = 0;                 // u_{t+1} (low byte) | its flags << 8 | dirty << 16 (cache not yet in the stack)
    int dsc = 0, Pdsc = 0;      // discrepancies on the path above level t, and above level t+1
    int my_root = -1;           // one-wave variant: the stored root the current item descends from
    unsigned c_eval = 0, c_node = 0, c_exp = 0, c_leaf = 0, c_items = 0;  // per lane; wave sums are 64-bit

    // add the wave's counters to the global ones (one atomic each) and clear them
    auto flush_counters = [&]() {
        unsigned long long s5[5] = {c_eval, c_node, c_exp, c_leaf, c_items};
#pragma unroll
        for (int q = 0; q < 5; ++q)
            for (int o = 32; o >= 1; o >>= 1) s5[q] += __shfl_xor(s5[q], o, 64);
        if (lane == 0)
#pragma unroll
            for (int q = 0; q < 5; ++q) atomicAdd(&a.counters[q], s5[q]);
        c_eval = c_node = c_exp = c_leaf = c_items = 0;
    };
    auto enter_level = [&]() {  // level t freshly entered from above
        y = centre_sum(t, k, my_u, s_muc + s_coff[t]);
        z = zig_init(y, tz != 0);
        onedir = tz;
        dir = 1;
        u = z.u1;
        applied = 0;
    };
    auto advance = [&]() { u = onedir ? u + dir : zig_next(z, u); };

    if (tid == 0 && blockIdx.x == 0) atomicCAS(a.t_start, 0ull, wall_clock());

    for (;;) {
        // ================= rare work (at most every kInner iterations) =================
        // per-lane 32-bit counters are flushed long before they could wrap
        if (__ballot(c_eval > (1u << 30))) flush_counters();
        // finished items
        {
            const unsigned long long fm = __ballot(fin != 0);
            if (fm && lane == (__ffsll((long long)fm) - 1))
                atomicAdd((unsigned long long *)a.pending, (unsigned long long)(-(long long)__popcll(fm)));
            fin = 0;
        }
        // stop flag (first hit, time cap, error)
        {
            int stop = 0;
            if (lane == 0) {
                stop = ld_rlx(&a.flags[0]);  // guards no data
                if (!stop && a.deadline) {
                    const unsigned long long t0 = ld_rlx(a.t_start);
                    if (t0 && wall_clock() > t0 + a.deadline) {
                        atomicOr(&a.flags[2], 1);
                        atomicOr(&a.flags[0], 1);
                        stop = 1;
                    }
                }
            }
            if (__shfl(stop, 0, 64)) state = DONE;
        }
        // exact leaf test (Thm 1) and A x = d, integers only
        if (__ballot(leafpend != 0)) {
            bool ok = false;
            uint8_t *xs = a.leaf_x + (size_t)(blockIdx.x * BLOCK + tid) * (size_t)a.n;  // this walker's staging row
            if (leafpend && state == RUN) {
                // v = sum_i u_i b_i exactly, each coordinate once.  A solution
                // has v_n = +-r_max and, with that sign taken off, |v_j| <= r_max
                // (Thm 1); x_j = (v_j + r_max) / (2 c_j) is staged, then A x = d
                // is checked from the staged row.
                const int64_t rmax = a.rmax;
                my_u[k - 1] = (int8_t)u;  // u_0 joins the prefix for the reconstruction
                auto coord = [&](int j) -> int64_t {
                    int64_t sv = 0;
                    for (int i = 0; i < k; ++i) sv += (int64_t)my_u[k - 1 - i] * a.basis[(size_t)i * a.dim + j];
                    return sv;
                };
                const int64_t vn = coord(a.n);
                ok = vn == rmax || vn == -rmax;
                const int64_t sg = vn > 0 ? 1 : -1;
                for (int j = 0; j < a.n && ok; ++j) {
                    const int64_t sv = sg * coord(j);
                    const int64_t cj2 = 2 * (a.cvec ? a.cvec[j] : 1);
                    ok = sv <= rmax && sv >= -rmax && (sv + rmax) % cj2 == 0;
                    if (ok) xs[j] = (uint8_t)((sv + rmax) / cj2);
                }
                for (int mi = 0; mi < a.m && ok; ++mi) {
                    int64_t acc = 0;
                    for (int j = 0; j < a.n; ++j) acc += (int64_t)a.A[(size_t)mi * a.n + j] * (int64_t)xs[j];
                    ok = acc == a.d[mi];
                }
            }
            // verified rows: one slot range per wave (ballot and prefix count)
            const unsigned long long om = __ballot(ok);
            if (om) {
                const int leader = __ffsll((long long)om) - 1;
                unsigned long long base = 0;
                if (lane == leader) {
                    base = atomicAdd(a.n_found, (unsigned long long)__popcll(om));
                    if (a.mode == 1) {
                        atomicCAS(a.t_first, 0ull, wall_clock());
                        atomicOr(&a.flags[0], 1);
                    }
                }
                base = __shfl(base, leader, 64);
                if (ok) {
                    const unsigned long long slot =
                        base + (unsigned)__builtin_amdgcn_mbcnt_hi((unsigned)(om >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((unsigned)om, 0));
                    if ((int64_t)slot < a.cap) {
                        if (a.sol_u) {
                            int8_t *so = a.sol_u + (size_t)slot * k;
                            for (int i = 0; i < k; ++i) so[i] = my_u[k - 1 - i];
                        }
                        uint8_t *xo = a.x_out + (size_t)slot * a.n;
                        for (int j = 0; j < a.n; ++j) xo[j] = xs[j];
                    }
                }
            }
            if (leafpend && state == RUN) {
                my_u[k - 1] = 0;
                advance();
            }
            leafpend = 0;
        }
        // donation: split off the untried values of the highest open level
        // while lanes hold tickets beyond the last item (head > tail)
        {
            // Every busy lane gives away work at once, which leaves a backlog
            // and keeps items large; levels below k/6 hold too little work to be
            // worth the receiver's prefix recomputation.
            int want = 0;
            if (lane == 0) {
                const unsigned long long h = ld_rlx(a.head), tl = ld_rlx(a.tail);
                want = h > tl;
            }
            if (__shfl(want, 0, 64)) {
                bool cand = state == RUN && top > t && top >= k / 6;
                int D = top, un = 0, fD = 0, dD = 0;
                if (cand) {
                    double yD, lD;
                    int uD;
                    if (D == t + 1) {
                        yD = Py; lD = Pl; uD = (int8_t)(Pw & 0xFF); fD = (Pw >> 8) & 0xFF; dD = BUDGETED ? Pdsc : 0;
                    } else {
                        const double *e = stack_at(D);
                        yD = e[0]; lD = e[1]; fD = (int)e[2]; dD = BUDGETED ? (int)e[3] : 0;
                        uD = my_u[k - 1 - D];
                    }
                    const double bD = s_beta[D];
                    const int odD = fD & F_ONEDIR, drD = (fD & F_DIRPOS) ? 1 : -1;
                    const Zig zD = zig_init(yD, (fD & F_TZ) != 0);
                    un = odD ? uD + drD : zig_next(zD, uD);
                    if (BUDGETED && dD + disc_cost(zD, un, (fD & F_TZ) != 0, dcount) > budget) {
                        // the budget ends level D before its next value
                        top = D - 1;
                        cand = false;
                    } else {
                        const double l = partial_norm(add_rn((double)un, yD), bD, lD);
                        if (!(l <= bound)) {
                            // nothing untried left at level D: this is the failing
                            // evaluation that would end level D, so count it here
                            ++c_eval;
                            top = D - 1;
                            cand = false;
                        }
                    }
                }
                const unsigned long long dm = __ballot(cand);
                if (dm) {
                    const int cnt = __popcll(dm);
                    const int leader = __ffsll((long long)dm) - 1;
                    int valid = 0;
                    unsigned long long base = 0;
                    if (lane == leader) {
                        base = atomicAdd(a.tail, (unsigned long long)cnt);
                        const long long room = (long long)a.pool.cap - (long long)base;
                        valid = room <= 0 ? 0 : (room < cnt ? (int)room : cnt);
                        if (valid) atomicAdd((unsigned long long *)a.pending, (unsigned long long)valid);
                    }
                    base = __shfl(base, leader, 64);
                    valid = __shfl(valid, leader, 64);
                    const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(dm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)dm, 0));
                    if (cand && rank < valid) {
                        const int64_t slot = (int64_t)base + rank;
                        int8_t *pu = a.pool.u + slot * k;
                        for (int j = 0; j < k; ++j) pu[j] = j > D ? my_u[k - 1 - j] : (int8_t)0;
                        a.pool.meta[slot] = make_int4(D, un, fD & (F_ONEDIR | F_DIRPOS | F_TZ), dD);
                        if (!ALLROWS) a.pool.root[slot] = my_root;
                        __hip_atomic_store(&a.pool.ready[slot], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                        top = D - 1;
                    }
                }
            }
        }
        // tickets: one atomic per wave; ticket i is pool slot i
        {
            const bool need = state == NEED_ROOT;
            const unsigned long long mask = __ballot(need);
            if (mask) {
                const int leader = __ffsll((long long)mask) - 1;
                unsigned long long base = 0;
                if (lane == leader) base = atomicAdd(a.head, (unsigned long long)__popcll(mask));
                base = __shfl(base, leader, 64);
                if (need) {
                    ticket = (unsigned)base + (unsigned)__builtin_amdgcn_mbcnt_hi(
                                                  (unsigned)(mask >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0));
                    state = WAIT;
                }
            }
        }
        // waiting lanes take their item once its slot is filled
        if (__ballot(state == WAIT)) {
            bool take = false;
            if (state == WAIT) {
                if ((long long)ticket < a.nroots) {
                    take = true;
                } else {
                    take = (long long)ticket < a.pool.cap && ld_rlx(&a.pool.ready[ticket]) != 0;
                    if (!take && ld_rlx(a.pending) == 0) state = DONE;
                }
            }
            // a donated slot seen ready: synchronise with its release store
            // before reading it (once per wave)
            if (__ballot(take && (long long)ticket >= a.nroots)) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            // Item set-up.  Row updates of w are made by code that every lane
            // of the wave runs (with a zero coefficient where a lane has
            // nothing to add); the one-wave variant's load of a stored w is
            // the exception, written under the lane mask of the taking lanes
            // (it needs no registers beyond w's own that way).
            if (ALLROWS) {
                if (take) {
                    const long long it = ((long long)ticket < a.nroots && a.order) ? a.order[ticket] : (long long)ticket;
                    const int4 mt = a.pool.meta[it];
                    if (BUDGETED) dsc = mt.w;
                    const int8_t *pu = a.pool.u + it * k;
                    load_prefix(my_u, pu, k, mt.x);
                    top = mt.x;
                    t = k - 1;          // next prefix level to add
                    lpar = 0.0;         // partial norm of the prefix so far
                    Pw = (mt.y & 0xFF) | ((mt.z & 0xFF) << 8);  // continuation, kept until the level is entered
                    state = LOAD;
                }
                if (__ballot(take)) {
                    const double keep = take ? 0.0 : 1.0;
#pragma unroll
                    for (int q = 0; q < DIMP; ++q) w[q] *= keep;
                }
            } else {
            long long it = 0, src = 0;  // src: the root whose stored w and norm the item starts from
            int T = 0, mflags = 0, mstart = 0;
            bool from_root = false, anchored = false;
            if (take) {
                it = ((long long)ticket < a.nroots && a.order) ? a.order[ticket] : (long long)ticket;
                const int4 mt = a.pool.meta[it];
                T = mt.x;
                mstart = mt.y;
                mflags = mt.z;
                if (BUDGETED) dsc = mt.w;
                const int8_t *pu = a.pool.u + it * k;
                load_prefix(my_u, pu, k, T);
                from_root = it < a.nroots;
                if (from_root) {
                    src = it;
                } else {  // a donated item below a stored root, or one with none above it
                    const int r = a.pool.root[it];
                    anchored = r >= 0;
                    src = anchored ? r : 0;
                }
                my_root = (from_root || anchored) ? (int)src : -1;
            }
            // a root from root generation, or the root a donated item descends
            // from: w and the partial norm at the roots' level are stored
            const bool stored = take && (from_root || anchored);
            double l = stored ? a.root_l[src] : 0.0;
            // The stored vector goes straight into w's registers: the loads
            // are written under the lane mask of the lanes that take one, so
            // they need no other registers and all of them can be in flight
            // at once.  Column rot + q is at pa + q wc before the wrap and at
            // pa + (q - DIMP) wc after it (one per-lane pointer, a uniform
            // stride).
            if (stored) {
                const int64_t wc = a.root_wcap;
                const double *pa = a.root_w + src + (int64_t)rot * wc;
                const int wrap_at = DIMP - rot;  // first register whose column wraps
#pragma unroll
                for (int q = 0; q < DIMP; ++q) w[q] = pa[(int64_t)(q < wrap_at ? q : q - DIMP) * wc];
            } else if (take) {
#pragma unroll
                for (int q = 0; q < DIMP; ++q) w[q] = 0.0;
            }
            // A donated item below a stored root adds the levels between the
            // roots' level and its own in the inner loop (state LOAD, one level
            // per iteration, rows in LDS), as the two-wave variant does.  One
            // with no stored root above it adds its whole prefix here, top
            // level first.  Either way these are the fused multiply-adds of root
            // generation in the same order, so w is the same.
            const bool pref = take && !from_root && !anchored;
            for (int j = k - 1; j >= 1; --j) {
                const bool act = pref && j > T;
                if (!__ballot(act)) break;
                double xj = 0.0;
                if (act) {
                    const double yj = centre_sum(j, k, my_u, s_muc + s_coff[j]);
                    xj = add_rn((double)my_u[k - 1 - j], yj);
                    l = partial_norm(xj, s_beta[j], l);
                }
                const double *gr = (j < L ? s_bh : a.g_bh) + (size_t)j * S + rot;
#pragma unroll
                for (int q = 0; q < DIMP; q += 2) {
                    const double2 b = *reinterpret_cast<const double2 *>(gr + q);
                    w[q] = fma(xj, b.x, w[q]);
                    w[q + 1] = fma(xj, b.y, w[q + 1]);
                }
            }
            if (take) {
                lpar = l;
                top = T;
                if (anchored && a.root_level - 1 > T) {
                    t = a.root_level - 1;  // next prefix level to add
                    Pw = (mstart & 0xFF) | ((mflags & 0xFF) << 8);  // continuation, kept until the level is entered
                    state = LOAD;
                } else {
                    t = T;
                    tz = (mflags & F_TZ) ? 1 : 0;
                    bt = s_beta[T];
                    enter_level();
                    if (!(mflags & F_FRESH)) {
                        u = mstart;
                        onedir = mflags & F_ONEDIR;
                        dir = (mflags & F_DIRPOS) ? 1 : -1;
                    }
                    fex = 0;
                    Pw = 0;
                    state = RUN;
                }
            }
            }
        }
        if (__ballot(state != DONE) == 0) break;
        if (__ballot(state == RUN || state == LOAD) == 0) {
            __builtin_amdgcn_s_sleep(32);  // the whole wave is waiting: back off
            continue;
        }

        // ================= inner loop: one row update per lane per iteration =================
#pragma unroll 1
        for (int it = 0; it < kInner; ++it) {
            // ---- control: at most two evaluations and one pop ----
            int row = 0;
            double coef = 0.0;
            bool node = false, popped = false;
            if (state == LOAD) {
                // one prefix level per iteration, top level first
                if (t > top) {
                    const double yj = centre_sum(t, k, my_u, s_muc + s_coff[t]);
                    const double xj = add_rn((double)my_u[k - 1 - t], yj);
                    lpar = partial_norm(xj, s_beta[t], lpar);
                    row = t;
                    coef = xj;
                    --t;
                }
                if (t == top) {  // the prefix is complete: enter the item's level
                    const int mstart = (int8_t)(Pw & 0xFF), mflags = (Pw >> 8) & 0xFF;
                    tz = (mflags & F_TZ) ? 1 : 0;
                    bt = s_beta[t];
                    enter_level();
                    if (!(mflags & F_FRESH)) {
                        u = mstart;
                        onedir = mflags & F_ONEDIR;
                        dir = (mflags & F_DIRPOS) ? 1 : -1;
                    }
                    fex = 0;
                    Pw = 0;
                    state = RUN;
                }
            } else
            while (state == RUN) {
                // a discrepancy budget ends the level at the first value whose
                // cost takes the path beyond it
                if (BUDGETED && !fex && dsc + disc_cost(z, u, tz != 0, dcount) > budget) fex = 1;
                if (!fex) {
                    const double x = add_rn((double)u, y);
                    const double l = partial_norm(x, bt, lpar);
                    ++c_eval;
                    if (l <= bound) {  // a NaN norm fails the test and ends the level
                        ++c_node;
                        if (t == 0) {  // a leaf: checked exactly in the rare-work pass
                            ++c_leaf;
                            leafpend = 1;
                            break;
                        }
                        node = true;
                        row = t;
                        coef = applied ? (double)(u - u_app) : x;
                        u_app = u;
                        applied = 1;
                        lcur = l;
                        break;
                    }
                }
                fex = 0;
                // level t is exhausted
                if (t == top) {
                    state = NEED_ROOT;
                    fin = 1;
                    ++c_items;
                    break;
                }
                if (popped) {
                    // a second pop would wait for the level state the first pop is
                    // still fetching: pop in the next iteration instead
                    fex = 1;
                    break;
                }
                const bool revert = applied != 0;
                if (revert) {
                    row = t;
                    coef = -add_rn((double)u_app, y);
                }
                ++t;
                y = Py;
                lpar = Pl;
                bt = s_beta[t];
                u = (int8_t)(Pw & 0xFF);
                if (BUDGETED) dsc = Pdsc;
                const int Pf = (Pw >> 8) & 0xFF;
                onedir = Pf & F_ONEDIR;
                dir = (Pf & F_DIRPOS) ? 1 : -1;
                tz = (Pf & F_TZ) ? 1 : 0;
                z = zig_init(y, tz != 0);
                u_app = u;
                applied = 1;
                if (t + 1 <= top) {
                    const double *e = stack_at(t + 1);
                    Py = e[0];
                    Pl = e[1];
                    Pw = (my_u[k - 2 - t] & 0xFF) | (((int)e[2] & 0xFF) << 8);
                    if (BUDGETED) Pdsc = (int)e[3];
                }
                advance();
                popped = true;
                if (revert) break;
            }

            // ---- the row update, all lanes together (a lane without one adds
            // 0 x row 0, which leaves w as it is) ----
            double h;
            {
                const double *br = s_bh + (size_t)row * S + rot;
                double h0 = 0.0, h1 = 0.0;
#pragma unroll
                for (int j = 0; j < DIMP; j += 2) {
                    const double2 b = *reinterpret_cast<const double2 *>(br + j);
                    w[j] = fma(coef, b.x, w[j]);
                    w[j + 1] = fma(coef, b.y, w[j + 1]);
                    h0 += fabs(w[j]);
                    h1 += fabs(w[j + 1]);
                }
                h = h0 + h1;
            }

            // ---- Hoelder test and the step that follows ----
            if (node) {
                const bool fail = hoelder && (lcur > (rmax_d * h) * hfac);
                if (fail) {
                    if (!onedir_cut) {
                        advance();
                    } else if (onedir) {
                        fex = 1;
                    } else {
                        u = zig_next(z, u);
                        onedir = 1;
                        dir = side_of(u, y);
                    }
                } else {
                    ++c_exp;
                    if (u > 127 || u < -127) {
                        atomicOr(&flagsp[1], 1);
                        atomicOr(&flagsp[0], 1);
                        state = DONE;
                    } else {
                        if ((Pw & 0x10000) && t + 1 <= top) {  // only a level first cached here needs writing
                            double *e = stack_at(t + 1);
                            e[0] = Py;
                            e[1] = Pl;
                            e[2] = (double)((Pw >> 8) & 0xFF);
                            if (BUDGETED) e[3] = (double)Pdsc;
                        }
                        if (BUDGETED) {
                            Pdsc = dsc;
                            dsc += disc_cost(z, u, tz != 0, dcount);
                        }
                        Py = y;
                        Pl = lpar;
                        Pw = (u & 0xFF) | (((onedir ? F_ONEDIR : 0) | (dir > 0 ? F_DIRPOS : 0) | (tz ? F_TZ : 0)) << 8) |
                             0x10000;
                        my_u[k - 1 - t] = (int8_t)u;
                        lpar = lcur;
                        tz = (tz && u == 0) ? 1 : 0;
                        --t;
                        bt = s_beta[t];
                        enter_level();
                    }
                }
            }
            // leave for the rare-work pass when a leaf waits for its check, when
            // eight lanes wait for work, or when no lane has any (waiting lanes
            // are served there too, but only every kInner iterations)
            if (__ballot(leafpend != 0) || __popcll(__ballot(state == NEED_ROOT)) >= 8 ||
                !__ballot(state == RUN || state == LOAD))
                break;
        }
    }
    flush_counters();
}

hipError_t launch_walk_prep(int k, int dim, int dimp, int block, const double *bhat, const double *mu,
                            double *g_bh, double *g_muc, int *g_coff, hipStream_t st) {
    hipLaunchKernelGGL(walk_prep_kernel, dim3(k), dim3(128), 0, st, k, dim, dimp, block, bhat, mu, g_bh, g_muc,
                       g_coff);
    return hipGetLastError();
}

int walk_muc_len(int k) { return walk_muc_offset(k, k - 1) + 8; }

template <int DIMP, int BLOCK, bool BUDGETED>
static hipError_t launch_variant(const WalkArgs &a, int num_cus, size_t lds, hipStream_t st) {
    hipError_t e = hipFuncSetAttribute((const void *)walk_kernel<DIMP, BLOCK, BUDGETED>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((walk_kernel<DIMP, BLOCK, BUDGETED>), dim3(num_cus), dim3(BLOCK), lds, st, a);
    return hipGetLastError();
}

template <int DIMP, int BLOCK>
static hipError_t launch_one(const WalkArgs &a, int num_cus, hipStream_t st) {
    // the two-wave variant keeps every row in LDS
    const size_t lds = walk_lds_bytes(DIMP, BLOCK, a.k, BLOCK == 512 ? a.k : a.L, a.muc_len);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    return a.budget >= 0 ? launch_variant<DIMP, BLOCK, true>(a, num_cus, lds, st)
                         : launch_variant<DIMP, BLOCK, false>(a, num_cus, lds, st);
}

int walk_max_level(int dimp, int k) {
    for (int L = k; L >= 1; --L)
        if (walk_lds_bytes(dimp, 256, k, L, walk_muc_len(k)) <= 160 * 1024) return L;
    return 0;
}

int walk_block_for(int dimp, int k, int L) {
    // two waves per SIMD where w is small enough, else one
    if (dimp <= 88 && walk_lds_bytes(dimp, 512, k, k, walk_muc_len(k)) <= 160 * 1024) return 512;
    return walk_lds_bytes(dimp, 256, k, L, walk_muc_len(k)) <= 160 * 1024 ? 256 : 0;
}

hipError_t launch_walk(const WalkArgs &a, int dimp, int block, int num_cus, hipStream_t st) {
#define MSP_CASE(D)                                                             \
    case D:                                                                     \
        if (block == 512 && D <= 88) return launch_one<D, 512>(a, num_cus, st); \
        if (block == 256) return launch_one<D, 256>(a, num_cus, st);            \
        return hipErrorInvalidValue;
    switch (dimp) {
        MSP_CASE(24) MSP_CASE(32) MSP_CASE(40) MSP_CASE(48) MSP_CASE(52) MSP_CASE(56) MSP_CASE(64)
        MSP_CASE(72) MSP_CASE(82) MSP_CASE(88) MSP_CASE(96) MSP_CASE(102) MSP_CASE(112) MSP_CASE(128)
        default: return hipErrorInvalidValue;
    }
#undef MSP_CASE
}

}  // namespace msp
