// Persistent subtree walker: Algorithm 1 (paper, Section 2) below the split
// level, one subtree per lane.
//
// Work distribution.  The grid is one or two workgroups per CU and stays
// resident; each lane that needs work takes the next subtree root from the
// queue (wave ballot + one atomic per wave + prefix count), walks that
// subtree to the end, and takes the next.  Walkers run until the queue is
// empty or, in first-solution mode, until a verified hit raises the stop flag.
//
// Per-lane state.  The projected vector w (Section 2: w^(t) = x_t b_hat_t +
// w^(t+1)) lives in DIMP registers.  It is updated incrementally: a new
// candidate at level t adds (u - u_applied) b_hat_t (an integer multiple) or
// x b_hat_t on first use of the level, and leaving level t subtracts the
// applied x_t b_hat_t.  Each loop iteration performs exactly one such row
// update per lane -- a node's update or a level's revert -- so all lanes run
// the expensive dim-length pass in lockstep; the cheap scalar control around
// it may diverge.
//
// LDS.  Rows b_hat_0..b_hat_{L-1} are stored with a padded stride S (a
// multiple of 16 doubles) and a wrap-around copy of their first 14 columns.
// Lane l keeps w in the column order rotated by r = 2 (l mod 8): register j
// holds column (j + r) mod DIMP and the pass reads row[r + j].  Eight lanes
// that read eight arbitrary rows then hit eight distinct 16-byte bank groups,
// so the 128-bit LDS reads are free of bank conflicts no matter which levels
// the lanes are on.  Only l1 norms and elementwise updates touch w, and both
// are independent of the column order.
// The strictly lower triangle of mu, beta, and an int8 stack of u values
// ([level][thread], for the centre sums and the leaf check) complete the LDS.
//
// Per-walker stack (HBM, one 32-byte entry per level: centre y, parent
// partial norm, zig-zag flags).  The state of the level above the current one
// is cached in registers, so popping a level never waits for memory; the
// entry above that is fetched while the walk continues.
#include "enum_rules.h"
#include "msp_internal.h"

namespace msp {

namespace {

enum : int { NEED_ROOT = 0, RUN = 1, DONE = 2 };
enum : int { K_NONE = 0, K_NODE = 1, K_REVERT = 2 };

constexpr int kRot = 2;  // rotation granule (columns): 128-bit reads

template <int DIMP>
struct Lds {
    static constexpr int S = ((DIMP + kRotMax + 15) / 16) * 16;
};

__device__ __forceinline__ unsigned long long wall_clock() { return wall_clock64(); }

__device__ __forceinline__ int load_flag(int *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace

template <int DIMP, int BLOCK>
__global__ void __launch_bounds__(BLOCK) walk_kernel(WalkArgs a) {
    constexpr int S = Lds<DIMP>::S;
    extern __shared__ __align__(16) unsigned char smem[];
    const int k = a.k, L = a.L, tid = threadIdx.x;
    double *s_bh = reinterpret_cast<double *>(smem);          // L x S
    double *s_mu = s_bh + (size_t)L * S;                      // row i (1..k-1) at i(i-1)/2
    double *s_beta = s_mu + (size_t)k * (k - 1) / 2;          // L (padded to even)
    int8_t *s_u = reinterpret_cast<int8_t *>(s_beta + ((L + 1) & ~1));  // k x BLOCK

    for (int idx = tid; idx < L * S; idx += BLOCK) {
        const int t = idx / S, p = idx - t * S;
        double v = 0.0;
        if (p < DIMP + kRotMax) {
            const int c = p < DIMP ? p : p - DIMP;
            if (c < a.dim) v = a.bhat[(size_t)t * a.dim + c];
        }
        s_bh[idx] = v;
    }
    for (int i = 1; i < k; ++i)
        for (int j = tid; j < i; j += BLOCK) s_mu[i * (i - 1) / 2 + j] = a.mu[(size_t)i * k + j];
    for (int t = tid; t < L; t += BLOCK) s_beta[t] = a.beta[t];
    for (int idx = tid; idx < k * BLOCK; idx += BLOCK) s_u[idx] = 0;
    __syncthreads();

    const int lane = tid & 63;
    const int rot = kRot * (lane & 7);
    const int64_t walker = (int64_t)blockIdx.x * BLOCK + tid;
    double *stk = a.stack + walker * (int64_t)k * 4;
    const int ws = DIMP + kWsTail;

    double w[DIMP];
#pragma unroll
    for (int j = 0; j < DIMP; ++j) w[j] = 0.0;

    int state = NEED_ROOT, fex = 0;
    int t = 0, u = 0, onedir = 0, dir = 1, tz = 0, applied = 0, u_app = 0;
    Zig z{0, 1};
    double y = 0.0, lpar = 0.0, lcur = 0.0;
    double Py = 0.0, Pl = 0.0;  // cached state of level t+1
    int Pf = 0;
    unsigned long long c_eval = 0, c_node = 0, c_exp = 0, c_leaf = 0, c_roots = 0;
    unsigned iter = 0;
    unsigned long long t_end = 0;
    if (lane == 0) {
        const unsigned long long t0 = wall_clock();
        if (tid == 0 && blockIdx.x == 0) atomicCAS(a.t_start, 0ull, t0);
        t_end = a.deadline ? t0 + a.deadline : 0;
    }

    // centre of level t from the u stack (levels > t), then the zig-zag start
    auto enter_level = [&]() {
        double yy = 0.0;
        for (int i = k - 1; i > t; --i)
            yy = add_rn(yy, mul_rn((double)s_u[i * BLOCK + tid], s_mu[i * (i - 1) / 2 + t]));
        y = yy;
        z = zig_init(y, tz != 0);
        onedir = tz;
        dir = 1;
        u = z.u1;
        applied = 0;
    };
    auto advance = [&]() { u = onedir ? u + dir : zig_next(z, u); };

    for (;;) {
        if ((iter++ & 63u) == 0) {
            int stop = 0;
            if (lane == 0) {
                stop = load_flag(&a.flags[0]);
                if (!stop && t_end && wall_clock() > t_end) {
                    atomicOr(&a.flags[2], 1);
                    atomicOr(&a.flags[0], 1);
                    stop = 1;
                }
            }
            stop = __shfl(stop, 0, 64);
            if (stop) state = DONE;
        }
        // ---- take roots (converged) ----
        const bool need = state == NEED_ROOT;
        const unsigned long long mask = __ballot(need);
        if (mask) {
            const int leader = __ffsll((long long)mask) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(a.qhead, (unsigned long long)__popcll(mask));
            base = __shfl(base, leader, 64);
            if (need) {
                const unsigned long long my = base + __popcll(mask & ((1ull << lane) - 1ull));
                if (my < (unsigned long long)a.nroots) {
                    const int64_t r = a.order ? a.order[my] : (int64_t)my;
                    const int8_t *pu = a.roots.u + r * k;
                    for (int i = L; i < k; ++i) s_u[i * BLOCK + tid] = pu[i];
                    const double *pw = a.roots.w + r * ws + rot;
#pragma unroll
                    for (int j = 0; j < DIMP; j += 2) {
                        const double2 v = *reinterpret_cast<const double2 *>(pw + j);
                        w[j] = v.x;
                        w[j + 1] = v.y;
                    }
                    lpar = a.roots.l[r];
                    tz = a.roots.tz[r];
                    t = L - 1;
                    enter_level();
                    fex = 0;
                    state = RUN;
                    ++c_roots;
                } else {
                    state = DONE;
                }
            }
        }
        if (__ballot(state != DONE) == 0) break;

        // ---- control: find this lane's row update ----
        int kind = K_NONE, row = 0;
        double coef = 0.0;
        unsigned guard = 0;
        while (state == RUN) {
            if (++guard > (1u << 20)) {  // no valid step sequence is this long: internal error
                atomicOr(&a.flags[3], 1);
                atomicOr(&a.flags[0], 1);
                state = DONE;
                break;
            }
            if (!fex) {
                const double x = add_rn((double)u, y);
                const double l = partial_norm(x, s_beta[t], lpar);
                ++c_eval;
                if (l <= a.bound) {  // a NaN norm fails the test and ends the level
                    ++c_node;
                    if (t == 0) {
                        ++c_leaf;
                        // exact leaf test (Thm 1) and A x = d, integers only
                        bool ok = true;
                        int64_t vn = 0;
                        {
                            int64_t s = (int64_t)u * a.basis[a.n];
                            for (int i = 1; i < k; ++i) s += (int64_t)s_u[i * BLOCK + tid] * a.basis[(size_t)i * a.dim + a.n];
                            vn = s;
                        }
                        if (vn != 1 && vn != -1) ok = false;
                        if (ok) {
                            for (int mi = 0; mi < a.m && ok; ++mi) {
                                int64_t acc = 0;
                                for (int j = 0; j < a.n; ++j) {
                                    int64_t s = (int64_t)u * a.basis[j];
                                    for (int i = 1; i < k; ++i)
                                        s += (int64_t)s_u[i * BLOCK + tid] * a.basis[(size_t)i * a.dim + j];
                                    s *= vn;
                                    if (s != 1 && s != -1) { ok = false; break; }
                                    if (s == 1) acc += a.A[(size_t)mi * a.n + j];
                                }
                                if (ok && acc != a.d[mi]) ok = false;
                            }
                        }
                        if (ok) {
                            const unsigned long long slot = atomicAdd(a.n_found, 1ull);
                            if ((int64_t)slot < a.cap) {
                                uint8_t *xo = a.x_out + (size_t)slot * a.n;
                                for (int j = 0; j < a.n; ++j) {
                                    int64_t s = (int64_t)u * a.basis[j];
                                    for (int i = 1; i < k; ++i)
                                        s += (int64_t)s_u[i * BLOCK + tid] * a.basis[(size_t)i * a.dim + j];
                                    xo[j] = (uint8_t)((s * vn + 1) / 2);
                                }
                            }
                            if (a.mode == 1) {
                                atomicCAS(a.t_first, 0ull, wall_clock());
                                atomicOr(&a.flags[0], 1);
                            }
                        }
                        advance();
                        continue;
                    }
                    kind = K_NODE;
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
            if (t == L - 1) {
                state = NEED_ROOT;
                break;
            }
            if (applied) {
                kind = K_REVERT;
                row = t;
                coef = -add_rn((double)u_app, y);
            }
            ++t;
            y = Py;
            lpar = Pl;
            onedir = Pf & 1;
            dir = (Pf & 2) ? 1 : -1;
            tz = (Pf >> 2) & 1;
            z = zig_init(y, tz != 0);
            u = s_u[t * BLOCK + tid];
            u_app = u;
            applied = 1;
            if (t + 1 <= L - 1) {
                const double *e = stk + (size_t)(t + 1) * 4;
                Py = e[0];
                Pl = e[1];
                Pf = (int)e[2];
            }
            advance();
            if (kind == K_REVERT) break;
        }

        // ---- the row update, all lanes together ----
        double h = 0.0;
        if (__ballot(kind != K_NONE)) {
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
        if (kind == K_NODE) {
            const bool fail = a.hoelder && (lcur > h * a.hfac);
            if (fail) {
                if (!a.onedir) {
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
                    atomicOr(&a.flags[1], 1);
                    atomicOr(&a.flags[0], 1);
                    state = DONE;
                } else {
                    if (t + 1 <= L - 1) {
                        double *e = stk + (size_t)(t + 1) * 4;
                        e[0] = Py;
                        e[1] = Pl;
                        e[2] = (double)Pf;
                    }
                    Py = y;
                    Pl = lpar;
                    Pf = onedir | (dir > 0 ? 2 : 0) | (tz << 2);
                    s_u[t * BLOCK + tid] = (int8_t)u;
                    lpar = lcur;
                    tz = (tz && u == 0) ? 1 : 0;
                    --t;
                    enter_level();
                }
            }
        }
    }

    // counters: one atomic per wave
    for (int o = 32; o >= 1; o >>= 1) {
        c_eval += __shfl_xor(c_eval, o, 64);
        c_node += __shfl_xor(c_node, o, 64);
        c_exp += __shfl_xor(c_exp, o, 64);
        c_leaf += __shfl_xor(c_leaf, o, 64);
        c_roots += __shfl_xor(c_roots, o, 64);
    }
    if (lane == 0) {
        atomicAdd(&a.counters[0], c_eval);
        atomicAdd(&a.counters[1], c_node);
        atomicAdd(&a.counters[2], c_exp);
        atomicAdd(&a.counters[3], c_leaf);
        atomicAdd(&a.counters[4], c_roots);
    }
}

size_t walk_lds_bytes(int dimp, int block, int k, int L) {
    const int S = ((dimp + kRotMax + 15) / 16) * 16;
    return sizeof(double) * ((size_t)L * S + (size_t)k * (k - 1) / 2 + (size_t)((L + 1) & ~1)) +
           (size_t)k * block;
}

template <int DIMP, int BLOCK>
static hipError_t launch_one(const WalkArgs &a, int num_cus, hipStream_t st) {
    const size_t lds = walk_lds_bytes(DIMP, BLOCK, a.k, a.L);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)walk_kernel<DIMP, BLOCK>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int per_cu = lds * 2 <= 160 * 1024 ? 2 : 1;
    hipLaunchKernelGGL((walk_kernel<DIMP, BLOCK>), dim3(num_cus * per_cu), dim3(BLOCK), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_walk(const WalkArgs &a, int dimp, int block, int num_cus, hipStream_t st) {
    if (block != 256) return hipErrorInvalidValue;
    switch (dimp) {
#define MSP_CASE(D) \
    case D: return launch_one<D, 256>(a, num_cus, st);
        MSP_CASE(24) MSP_CASE(32) MSP_CASE(40) MSP_CASE(48) MSP_CASE(52) MSP_CASE(56) MSP_CASE(64)
        MSP_CASE(72) MSP_CASE(82) MSP_CASE(88) MSP_CASE(96) MSP_CASE(102) MSP_CASE(112) MSP_CASE(128)
#undef MSP_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace msp
