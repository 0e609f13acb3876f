// C ABI of libmsp (declared in include/msp.h): argument checks, the
// context's device workspace, and the sequence of kernel launches for each
// call.  No arithmetic of the method happens on the host: every step runs in
// the kernels of gs.hip, rootgen.hip, walk.hip, lll.hip and order.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "../../include/msp.h"
#include "expand_thin.h"
#include "msp_internal.h"

using namespace msp;

namespace {

struct Buf {
    void *p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes) {
        if (bytes <= cap) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            cap = 0;
        }
        size_t nb = std::max<size_t>(bytes, 256);
        hipError_t e = hipMalloc(&p, nb);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        cap = nb;
        return hipSuccess;
    }
    // like ensure(), but keeps the first `cap` bytes (copied on the stream)
    hipError_t grow(size_t bytes, hipStream_t st) {
        if (bytes <= cap) return hipSuccess;
        size_t nb = std::max<size_t>(bytes, 2 * cap);
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, nb);
        if (e != hipSuccess) return e;
        if (p) {
            e = hipMemcpyAsync(q, p, cap, hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) {
                (void)hipFree(q);
                return e;
            }
            (void)hipFree(p);
        }
        p = q;
        cap = nb;
        return hipSuccess;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <class T>
    T *as() const {
        return reinterpret_cast<T *>(p);
    }
};

struct FrontierBuf {
    Buf u, w, l, tz, dsc;
    int64_t cap = 0;
    hipError_t ensure(int64_t n, int k, int ws) {
        hipError_t e;
        if ((e = u.ensure((size_t)n * k)) != hipSuccess) return e;
        if ((e = w.ensure((size_t)n * ws * sizeof(double))) != hipSuccess) return e;
        if ((e = l.ensure((size_t)n * sizeof(double))) != hipSuccess) return e;
        if ((e = tz.ensure((size_t)n)) != hipSuccess) return e;
        if ((e = dsc.ensure((size_t)n)) != hipSuccess) return e;
        cap = n;
        return hipSuccess;
    }
    Frontier view() const {
        return Frontier{u.as<int8_t>(), w.as<double>(), l.as<double>(), tz.as<uint8_t>(), dsc.as<uint8_t>(), cap};
    }
    void release() {
        u.release();
        w.release();
        l.release();
        tz.release();
        dsc.release();
        cap = 0;
    }
};

// Small device-side control block, one allocation.
struct Ctl {
    unsigned long long counters[8];  // evals nodes expansions leaves roots
    unsigned long long qhead;      // pool claim cursor
    unsigned long long qtail;      // pool append cursor
    long long pending;             // unfinished pool items
    unsigned long long n_found;
    unsigned long long t_first;
    unsigned long long t_start;
    int flags[8];                    // stop overflow timeout internal
    int gs_err;
    int pad;
    int64_t total;
    ThinOut thin;
};

}  // namespace

struct msp_ctx {
    int device = 0;
    int num_cus = 0;
    double wall_khz = 100000.0;
    Buf gs_bhat, gs_mu, gs_beta;
    FrontierBuf fr[3];
    Buf counts, offs;
    Buf stack;
    Buf ctl;
    Buf order;
    Buf lll_desc, lll_work, batch_basis;
    Buf g_bh, g_muc, g_coff;
    Buf pool_u, pool_meta, pool_ready, pool_root;
    Buf leaf_x;  // the walkers' leaf staging rows
    Buf box_d, box_r, box_basis, box_x, box_st;  // msp_solve_box: shifted problem and its rows
    long long last_lll_iters = 0;
    // tuned root counts (msp_autotune), keyed by (architecture, mode, m, n bucket)
    struct Tuned {
        std::string arch;
        int mode, m, nbucket, target_roots;
    };
    std::string arch;
    std::vector<Tuned> tuned;
    hipEvent_t ev[8] = {};
    // root orders
    Buf feat, key, key_out, idx_in, sort_tmp, scan_tmp;
    Buf left_u, left_meta, top_idx;  // refinement: stage leftovers, best-node indices
    Buf cvec, rmax;                  // bounded variables: c_j and r_max of the last bounds
    Buf bkz_out, bkz_save;           // BKZ status words and the LLL basis kept for a fallback
    Buf rs_A, rs_perm, rs_basis, rs_x;  // msp_solve_first: shuffled copies, their bases, a hit's rows
    // roots of the last enumeration (for tracing)
    int last_cur = 0, last_L = 0, last_k = 0, last_dim = 0, last_ws = 0, last_m = 0;
    int64_t last_np = 0;
    double last_R = 0.0;
    Buf sol_u, trace_x;
    // root-scoring model
    bool has_model = false;
    Buf w_master, w_q, adam_m, adam_v, step, partial, loss_acc, dev_loss, npos;
    Buf sh_keys, sh_keys_out, sh_idx, sh_perm, sh_tmp;
    hipStream_t aux = nullptr;
};

namespace {

int map_err(hipError_t e) {
    if (e == hipSuccess) return MSP_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return MSP_E_NOMEM;
    return MSP_E_DEVICE;
}

#define MSP_TRY(expr)                          \
    do {                                       \
        hipError_t _e = (expr);                \
        if (_e != hipSuccess) return map_err(_e); \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

}  // namespace

extern "C" {

int msp_params_default(msp_params *p) {
    if (!p) return MSP_E_ARG;
    p->N = 1024;
    p->delta = 0.99;
    p->eps = 1e-9;
    p->split_depth = -1;
    p->block = 0;
    p->target_roots = 0;
    p->hoelder = 1;
    p->onedir = 1;
    p->time_cap_ms = 0.0;
    p->refine = 0;
    p->refine_keep = 0;
    p->disc_budget = -1;
    p->bkz_block = 0;
    p->bkz_tours = 4;
    p->restarts = 1;
    p->restart_seed = 1;
    p->disc_count = 0;
    p->root_begin = 0;
    p->root_count = -1;
    return MSP_OK;
}

const char *msp_strerror(int code) {
    switch (code) {
        case MSP_OK: return "ok";
        case MSP_E_ARG: return "invalid argument";
        case MSP_E_RANK: return "rank of A is below m";
        case MSP_E_NOT_ISOLATED: return "scale N too small: kernel vectors not isolated";
        case MSP_E_OVERFLOW: return "integer bound exceeded";
        case MSP_E_CAPACITY: return "more solutions than the output capacity";
        case MSP_E_TIMEOUT: return "time cap reached";
        case MSP_E_DEVICE: return "HIP runtime error";
        case MSP_E_NOMEM: return "device memory allocation failed";
        case MSP_E_UNSUPPORTED: return "shape outside the compiled kernel variants";
        case MSP_E_NUMERIC: return "floating-point breakdown";
        default: return "unknown status";
    }
}

int msp_ctx_create(int device, msp_ctx **out) {
    if (!out) return MSP_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MSP_E_DEVICE;
    DeviceGuard g(device);
    msp_ctx *c = new (std::nothrow) msp_ctx();
    if (!c) return MSP_E_NOMEM;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return MSP_E_DEVICE;
    }
    c->num_cus = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    int rate = 0;
    if (hipDeviceGetAttribute(&rate, hipDeviceAttributeWallClockRate, device) == hipSuccess && rate > 0)
        c->wall_khz = rate;
    for (auto &e : c->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            msp_ctx_destroy(c);
            return MSP_E_DEVICE;
        }
    }
    if (c->ctl.ensure(sizeof(Ctl)) != hipSuccess) {
        msp_ctx_destroy(c);
        return MSP_E_NOMEM;
    }
    *out = c;
    return MSP_OK;
}

void msp_ctx_destroy(msp_ctx *c) {
    if (!c) return;
    DeviceGuard g(c->device);
    c->gs_bhat.release();
    c->gs_mu.release();
    c->gs_beta.release();
    c->fr[0].release();
    c->fr[1].release();
    c->fr[2].release();
    c->left_u.release();
    c->left_meta.release();
    c->top_idx.release();
    c->cvec.release();
    c->rmax.release();
    c->bkz_out.release();
    c->bkz_save.release();
    c->rs_A.release();
    c->rs_perm.release();
    c->rs_basis.release();
    c->rs_x.release();
    c->counts.release();
    c->offs.release();
    c->stack.release();
    c->ctl.release();
    c->order.release();
    c->lll_desc.release();
    c->lll_work.release();
    c->batch_basis.release();
    c->g_bh.release();
    c->g_muc.release();
    c->g_coff.release();
    c->pool_u.release();
    c->pool_meta.release();
    c->pool_ready.release();
    c->pool_root.release();
    c->leaf_x.release();
    for (Buf *b : {&c->box_d, &c->box_r, &c->box_basis, &c->box_x, &c->box_st}) b->release();
    for (Buf *b : {&c->feat, &c->key, &c->key_out, &c->idx_in, &c->sort_tmp, &c->scan_tmp, &c->sol_u, &c->trace_x, &c->w_master,
                   &c->w_q, &c->adam_m, &c->adam_v, &c->step, &c->partial, &c->loss_acc, &c->dev_loss, &c->npos,
                   &c->sh_keys, &c->sh_keys_out, &c->sh_idx, &c->sh_perm, &c->sh_tmp})
        b->release();
    if (c->aux) (void)hipStreamDestroy(c->aux);
    for (auto &e : c->ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
}

int msp_gram_schmidt(msp_ctx *c, int k, int dim, const int64_t *basis_dev, double *bhat_dev, double *mu_dev,
                     double *beta_dev, void *stream) {
    if (!c || !basis_dev || !bhat_dev || !mu_dev || !beta_dev) return MSP_E_ARG;
    if (k < 1 || dim < 1 || k > dim || dim > MSP_MAX_N + 1) return MSP_E_ARG;
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    Ctl *ctl = c->ctl.as<Ctl>();
    MSP_TRY(hipMemsetAsync(&ctl->gs_err, 0, sizeof(int), st));
    GsArgs a{k, dim, basis_dev, bhat_dev, mu_dev, beta_dev, &ctl->gs_err};
    MSP_TRY(launch_gram_schmidt(a, st));
    int err = 0;
    MSP_TRY(hipMemcpyAsync(&err, &ctl->gs_err, sizeof(int), hipMemcpyDeviceToHost, st));
    MSP_TRY(hipStreamSynchronize(st));
    return err ? MSP_E_NUMERIC : MSP_OK;
}

}  // extern "C"

static int enumerate_impl(msp_ctx *c, int m, int n, const int32_t *A_dev, const int64_t *d_dev,
                          const int64_t *basis_dev, int k, int mode, int order, const msp_params *pin, uint8_t *x_dev,
                          int64_t cap, int64_t *n_found, msp_stats *stats, void *stream, int8_t *sol_u = nullptr,
                          const int64_t *cvec = nullptr, long long rmax = 1, bool gs_ready = false) {
    auto t_call = std::chrono::steady_clock::now();
    if (!c || !A_dev || !d_dev || !basis_dev || !n_found || (cap > 0 && !x_dev) || cap < 0) return MSP_E_ARG;
    if (m < 1 || n < 1 || m > n || n > MSP_MAX_N || k != n - m + 1) return MSP_E_ARG;
    if (mode != MSP_ALL && mode != MSP_FIRST) return MSP_E_ARG;
    if (order != MSP_PLAIN && order != MSP_LEARNED && order != MSP_DISCREPANCY) return MSP_E_ARG;
    if (order == MSP_LEARNED && !c->has_model) return MSP_E_ARG;
    msp_params p;
    msp_params_default(&p);
    if (pin) p = *pin;
    if (!(p.eps >= 0.0) || p.split_depth < -1 || p.split_depth > k - 1) return MSP_E_ARG;
    if (p.refine < -1 || p.refine_keep < 0 || p.target_roots < 0 || p.disc_budget > 255) return MSP_E_ARG;
    if (p.disc_count != 0 && p.disc_count != 1) return MSP_E_ARG;
    if (p.root_begin < 0 || p.root_count < -1) return MSP_E_ARG;
    const bool ranged = p.root_begin != 0 || p.root_count >= 0;
    *n_found = 0;
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    const int dim = n + 1;
    const int dimp = dimp_for(dim);
    if (dimp < 0) return MSP_E_UNSUPPORTED;
    const int ws = dimp;  // columns of a stored projected vector
    if (p.block != 0 && p.block != 256 && p.block != 512) return MSP_E_ARG;

    // ---- Gram-Schmidt (step 3) ----
    MSP_TRY(c->gs_bhat.ensure((size_t)k * dim * sizeof(double)));
    MSP_TRY(c->gs_mu.ensure((size_t)k * k * sizeof(double)));
    MSP_TRY(c->gs_beta.ensure((size_t)k * sizeof(double)));
    Ctl *ctl = c->ctl.as<Ctl>();
    MSP_TRY(hipMemsetAsync(ctl, 0, sizeof(Ctl), st));
    MSP_TRY(hipEventRecord(c->ev[0], st));
    // gs_ready: the caller ran this call's Gram-Schmidt on the same basis
    // before (the passes of one discrepancy search), and the buffers hold it
    if (!gs_ready) {
        GsArgs ga{k, dim, basis_dev, c->gs_bhat.as<double>(), c->gs_mu.as<double>(), c->gs_beta.as<double>(),
                  &ctl->gs_err};
        MSP_TRY(launch_gram_schmidt(ga, st));
    }
    MSP_TRY(hipEventRecord(c->ev[1], st));
    if (!gs_ready) {
        int gs_err = 0;
        MSP_TRY(hipMemcpyAsync(&gs_err, &ctl->gs_err, sizeof(int), hipMemcpyDeviceToHost, st));
        MSP_TRY(hipStreamSynchronize(st));
        if (gs_err) return MSP_E_NUMERIC;
    }

    const double R = (double)(n + 1) * (double)rmax * (double)rmax;  // (n+1) r_max^2 (Algorithm 1, step 4)
    const double bound = R * (1.0 + p.eps);
    const double hfac = 1.0 + p.eps;

    // ---- root generation: levels k-1 .. L breadth first ----
    // lanes of the walk kernel (two waves per SIMD where w is narrow enough)
    const int64_t walkers = (int64_t)c->num_cus * (dimp <= 88 && p.block != 256 ? 512 : 256);
    const bool ordered_first = mode == MSP_FIRST && order != MSP_PLAIN;
    const bool refine = ordered_first && p.refine != 0;
    const int max_stages = p.refine > 0 ? p.refine : 64;
    const int64_t keep = p.refine_keep > 0 ? p.refine_keep : walkers;
    // The walker splits work dynamically, so for an exhaustive walk a few
    // roots per lane suffice.  A first-solution search wants small subtrees:
    // a lane walks its subtree alone until the roots run out, so the root
    // order only pays off when each subtree is a short walk (refinement gets
    // there in stages, from a smaller first frontier).
    const int64_t target = p.target_roots > 0 ? p.target_roots
                           : refine             ? 16 * walkers
                           : mode == MSP_FIRST  ? 64 * walkers
                                                : std::max<int64_t>(2 * walkers, 4096);
    const int64_t fcap = std::max<int64_t>(4 * std::max<int64_t>(target, keep), 1 << 16);
    MSP_TRY(c->fr[0].ensure(fcap, k, ws));
    MSP_TRY(c->fr[1].ensure(fcap, k, ws));
    if (refine) MSP_TRY(c->fr[2].ensure(fcap, k, ws));
    MSP_TRY(c->counts.ensure((size_t)fcap * sizeof(int64_t)));
    MSP_TRY(c->offs.ensure((size_t)fcap * sizeof(int64_t)));
    {
        size_t tb = 0;
        MSP_TRY(launch_scan(nullptr, &tb, c->counts.as<int64_t>(), c->offs.as<int64_t>(), fcap, &ctl->total, st));
        MSP_TRY(c->scan_tmp.ensure(tb > 0 ? tb : 1));
    }
    MSP_TRY(hipEventRecord(c->ev[2], st));
    MSP_TRY(launch_frontier_init(c->fr[0].view(), k, ws, st));
    // the walker keeps rows b_hat_0 .. b_hat_{L-1} in LDS: split at least this deep
    const int L_fit = walk_max_level(dimp, k);
    if (L_fit < 1) return MSP_E_UNSUPPORTED;

    // Expand the frontier in fr[cur] (np nodes of level L) one level at a
    // time into fr[other], swapping, until the rule says done or level 1.  A
    // level that would not fit the frontier buffers is not taken.  While a
    // level has at most kThinMax parents, one launch takes the levels (one
    // host round trip for all of them); wider levels take a count launch,
    // a scan, a host read of the total and a write launch each.
    bool capped = false;  // a level was left unexpanded for lack of frontier room
    auto expand = [&](int &cur, int other, int64_t &np, int &L, const ThinRule &rule) -> int {
        ExpandArgs base{};  // what every level shares
        base.k = k;
        base.dim = dim;
        base.dimp = dimp;
        base.ws = ws;
        base.bhat = c->gs_bhat.as<double>();
        base.mu = c->gs_mu.as<double>();
        base.beta = c->gs_beta.as<double>();
        base.offs = c->offs.as<int64_t>();
        base.counts = c->counts.as<int64_t>();
        base.bound = bound;
        base.hfac = hfac;
        base.rmax = (double)rmax;
        base.budget = p.disc_budget;
        base.disc_count = p.disc_count;
        base.hoelder = p.hoelder;
        base.onedir = p.onedir;
        base.counters = ctl->counters;
        base.flags = ctl->flags;
        while (L - 1 >= 1 && !thin_done(rule, np, L)) {
            if (np >= 1 && np <= kThinMax) {
                ThinArgs ta;
                std::memset(&ta, 0, sizeof(ta));
                ta.e = base;
                ta.fr[0] = c->fr[cur].view();
                ta.fr[1] = c->fr[other].view();
                ta.np = np;
                ta.L = L;
                ta.fcap = fcap;
                ta.rule = rule;
                ta.out = &ctl->thin;
                MSP_TRY(launch_expand_thin(ta, st));
                ThinOut o;
                MSP_TRY(hipMemcpyAsync(&o, &ctl->thin, sizeof(o), hipMemcpyDeviceToHost, st));
                MSP_TRY(hipStreamSynchronize(st));
                if (o.cur) std::swap(cur, other);
                const bool moved = o.L != L;
                np = o.np;
                L = o.L;
                if (o.capped) {
                    capped = true;
                    break;
                }
                if (np == 0) break;
                // it stopped at the rule, at level 1 or at a level too wide for it
                if (moved) continue;
            }
            const int t = L - 1;
            ExpandArgs ea = base;
            ea.t = t;
            ea.par = c->fr[cur].view();
            ea.np = np;
            ea.ch = c->fr[other].view();
            MSP_TRY(launch_expand_count(ea, st));
            size_t tb = c->scan_tmp.cap;
            MSP_TRY(launch_scan(c->scan_tmp.p, &tb, c->counts.as<int64_t>(), c->offs.as<int64_t>(), np, &ctl->total,
                                st));
            int64_t total = 0;
            MSP_TRY(hipMemcpyAsync(&total, &ctl->total, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            MSP_TRY(hipStreamSynchronize(st));
            if (total > fcap) {  // cannot hold this level: split above it
                capped = true;
                break;
            }
            MSP_TRY(launch_expand_write(ea, st));
            std::swap(cur, other);
            np = total;
            L = t;
            if (np == 0) break;
        }
        return MSP_OK;
    };

    int cur = 0;
    int64_t np = 1;
    int L = k;
    {
        ThinRule rule{};
        rule.k = k;
        if (p.split_depth >= 0) {  // fixed split depth
            rule.kind = 0;
            rule.depth = p.split_depth;
        } else {  // enough roots, and deep enough for the walker's LDS rows
            rule.kind = 1;
            rule.target = target;
            rule.lb = L_fit;
        }
        int rc = expand(cur, 1, np, L, rule);
        if (rc != MSP_OK) return rc;
    }
    const int L0 = L;  // highest level of any walked item: the walker's LDS rows
    // The automatic split expanded every level down to 1 and still found fewer
    // roots than it aimed for: the whole tree is small (a few nodes per root
    // below level 1).  Then a grid of about two lanes per root walks it; a
    // full grid would leave most lanes waiting while busy lanes split tiny
    // items for them, each paying a prefix rebuild.
    const bool small_tree = p.split_depth < 0 && L == 1 && np < target && !capped;
    const int64_t np0 = np;
    MSP_TRY(hipEventRecord(c->ev[3], st));
    c->last_cur = cur;
    c->last_np = np;
    c->last_L = L;
    c->last_k = k;
    c->last_dim = dim;
    c->last_ws = ws;
    c->last_m = m;
    c->last_R = R;

    // ---- root order for first-solution search ----
    // Order the np records of frontier fr[f] (level Lf) best first into c->order.
    auto order_frontier = [&](int f, int64_t nrec, int Lf) -> int {
        MSP_TRY(c->feat.ensure((size_t)nrec * kNumFeat * sizeof(float)));
        MSP_TRY(c->key.ensure((size_t)nrec * sizeof(float)));
        MSP_TRY(c->key_out.ensure((size_t)nrec * sizeof(float)));
        MSP_TRY(c->idx_in.ensure((size_t)nrec * sizeof(int64_t)));
        MSP_TRY(c->order.ensure((size_t)nrec * sizeof(int64_t)));
        FeatArgs fa{k, dim, m, Lf, ws, c->fr[f].view(), nrec, c->gs_mu.as<double>(), c->gs_beta.as<double>(), R,
                    c->feat.as<float>()};
        MSP_TRY(launch_root_features(fa, st));
        if (order == MSP_LEARNED)
            MSP_TRY(launch_mlp_score(c->w_q.as<float>(), c->feat.as<float>(), nrec, c->key.as<float>(), st));
        else
            MSP_TRY(launch_disc_keys(c->feat.as<float>(), nrec, k - Lf, c->key.as<float>(), st));
        size_t tb = 0;
        MSP_TRY(sort_scores_desc(nullptr, &tb, c->key.as<float>(), c->key_out.as<float>(), c->idx_in.as<int64_t>(),
                                 c->order.as<int64_t>(), nrec, st));
        MSP_TRY(c->sort_tmp.ensure(tb));
        tb = c->sort_tmp.cap;
        MSP_TRY(sort_scores_desc(c->sort_tmp.p, &tb, c->key.as<float>(), c->key_out.as<float>(),
                                 c->idx_in.as<int64_t>(), c->order.as<int64_t>(), nrec, st));
        return MSP_OK;
    };
    const bool ordered = order != MSP_PLAIN && np > 1;
    int stages = 0;
    std::vector<std::pair<int64_t, int64_t>> left;  // (offset, count) of each stage's leftovers
    int64_t nleft = 0;
    if (ordered) {
        MSP_TRY(hipEventRecord(c->ev[6], st));
        int rc = order_frontier(cur, np, L);
        if (rc != MSP_OK) return rc;
        if (refine) {
            // refine until the walked subtrees are a few levels deep
            const int L_stop = std::max(2, k / 16);
            while (stages < max_stages && L > L_stop && np > keep) {
                // the rest of this frontier becomes work items, walked after
                // everything the refinement of the best nodes produces
                const int64_t rest = np - keep;
                MSP_TRY(c->left_u.grow((size_t)(nleft + rest) * k, st));
                MSP_TRY(c->left_meta.grow((size_t)(nleft + rest) * sizeof(int4), st));
                MSP_TRY(launch_frontier_items(c->fr[cur].view(), c->order.as<int64_t>() + keep, rest, k, L,
                                              c->left_u.as<int8_t>() + nleft * k, c->left_meta.as<int4>() + nleft,
                                              st));
                left.emplace_back(nleft, rest);
                nleft += rest;
                // the best nodes, back in depth-first order, as the next frontier
                MSP_TRY(c->top_idx.ensure((size_t)keep * sizeof(int64_t)));
                size_t tb = 0;
                MSP_TRY(sort_idx_asc(nullptr, &tb, c->order.as<int64_t>(), c->top_idx.as<int64_t>(), keep, st));
                MSP_TRY(c->sort_tmp.ensure(tb));
                tb = c->sort_tmp.cap;
                MSP_TRY(sort_idx_asc(c->sort_tmp.p, &tb, c->order.as<int64_t>(), c->top_idx.as<int64_t>(), keep, st));
                const int nxt = (cur + 1) % 3, oth = (cur + 2) % 3;
                MSP_TRY(launch_gather_frontier(c->fr[cur].view(), c->top_idx.as<int64_t>(), 0, keep, c->fr[nxt].view(),
                                               k, ws, st));
                int a = nxt;
                int64_t n2 = keep;
                int L2 = L;
                ThinRule rule{};
                rule.kind = 2;  // enough roots, or as deep as the refinement goes
                rule.k = k;
                rule.target = target;
                rule.lb = L_stop;
                rc = expand(a, oth, n2, L2, rule);
                if (rc != MSP_OK) return rc;
                ++stages;
                const bool deeper = L2 < L;  // false: the next level would not fit the buffers
                cur = a;
                np = n2;
                L = L2;
                if (np > 1) {
                    rc = order_frontier(cur, np, L);
                    if (rc != MSP_OK) return rc;
                }
                if (!deeper || np == 0) break;
            }
        }
        MSP_TRY(hipEventRecord(c->ev[7], st));
    }
    const bool use_order = ordered && np > 1;

    // ---- optional range of root positions (checkpoint / resume, sharding):
    // the records at those positions of the walk order, gathered into fr[2] ----
    int wcur = cur;            // frontier holding the walked roots
    int64_t wnp = np;          // walked roots
    const int64_t *worder = use_order ? c->order.as<int64_t>() : nullptr;
    if (ranged) {
        if (refine) return MSP_E_ARG;
        const int64_t rb = std::min<int64_t>(p.root_begin, np);
        const int64_t rn = p.root_count < 0 ? np - rb : std::min<int64_t>(p.root_count, np - rb);
        MSP_TRY(c->fr[2].ensure(fcap, k, ws));
        MSP_TRY(launch_gather_frontier(c->fr[cur].view(), worder ? worder + rb : nullptr, rb, rn, c->fr[2].view(), k,
                                       ws, st));
        wcur = 2;
        wnp = rn;
        worder = nullptr;
        // only the call whose range starts at position 0 counts the levels
        // above the split, so the counters of a cover of the roots add up
        if (p.root_begin > 0) MSP_TRY(launch_fill_int(reinterpret_cast<int *>(ctl->counters), 16, 0, st));
    }

    // ---- subtree walk (levels L0-1 .. 0) ----
    int wblock = walk_block_for(dimp, k, L0);
    if (p.block != 0 && wblock != 0) wblock = std::min(wblock, p.block);
    if (wblock == 0) return MSP_E_UNSUPPORTED;
    const int muc_len = walk_muc_len(k);
    const int S = walk_row_stride(dimp, wblock);
    MSP_TRY(c->g_bh.ensure((size_t)k * S * sizeof(double)));
    MSP_TRY(c->g_muc.ensure((size_t)muc_len * sizeof(double)));
    MSP_TRY(c->g_coff.ensure((size_t)(k + 2) * sizeof(int)));
    MSP_TRY(launch_walk_prep(k, dim, dimp, wblock, c->gs_bhat.as<double>(), c->gs_mu.as<double>(), c->g_bh.as<double>(),
                             c->g_muc.as<double>(), c->g_coff.as<int>(), st));
    const int64_t nwalk = (int64_t)c->num_cus * wblock;
    MSP_TRY(c->stack.ensure((size_t)nwalk * k * 4 * sizeof(double)));
    MSP_TRY(c->leaf_x.ensure((size_t)nwalk * n));
    const int64_t ninit = wnp + nleft;  // roots with stored w, then prefix-only items
    const int64_t pcap = ninit + std::max<int64_t>(256 * nwalk, 1 << 22);
    if (pcap + nwalk >= (int64_t(1) << 31)) return MSP_E_UNSUPPORTED;  // walker tickets are 32-bit
    MSP_TRY(c->pool_u.ensure((size_t)pcap * k));
    MSP_TRY(c->pool_meta.ensure((size_t)pcap * sizeof(int4)));
    MSP_TRY(c->pool_ready.ensure((size_t)pcap * sizeof(int)));
    MSP_TRY(c->pool_root.ensure((size_t)pcap * sizeof(int)));
    Pool pool{c->pool_u.as<int8_t>(), c->pool_meta.as<int4>(), c->pool_ready.as<int>(), c->pool_root.as<int>(),
              pcap};
    if (ninit > 0) {
        MSP_TRY(launch_pool_init(c->fr[wcur].view(), wnp, k, L, pool, st));
        // leftovers of the refinement stages, latest stage first
        int64_t pos = np;
        for (size_t s = left.size(); s-- > 0;) {
            const int64_t off = left[s].first, cnt = left[s].second;
            MSP_TRY(hipMemcpyAsync(pool.u + pos * k, c->left_u.as<int8_t>() + off * k, (size_t)cnt * k,
                                   hipMemcpyDeviceToDevice, st));
            MSP_TRY(hipMemcpyAsync(pool.meta + pos, c->left_meta.as<int4>() + off, (size_t)cnt * sizeof(int4),
                                   hipMemcpyDeviceToDevice, st));
            pos += cnt;
        }
        MSP_TRY(launch_fill_int(pool.ready + np, nleft, 1, st));
        MSP_TRY(launch_fill_int(pool.root + np, nleft, -1, st));  // no stored root above them
        const unsigned long long qt = (unsigned long long)ninit;
        const long long pend = (long long)ninit;
        MSP_TRY(hipMemcpyAsync(&ctl->qtail, &qt, sizeof(qt), hipMemcpyHostToDevice, st));
        MSP_TRY(hipMemcpyAsync(&ctl->pending, &pend, sizeof(pend), hipMemcpyHostToDevice, st));
        WalkArgs wa{};
        wa.k = k;
        wa.dim = dim;
        wa.n = n;
        wa.m = m;
        wa.L = L0;
        wa.g_bh = c->g_bh.as<double>();
        wa.g_muc = c->g_muc.as<double>();
        wa.g_coff = c->g_coff.as<int>();
        wa.muc_len = muc_len;
        wa.beta = c->gs_beta.as<double>();
        wa.basis = basis_dev;
        wa.A = A_dev;
        wa.d = d_dev;
        wa.pool = pool;
        wa.nroots = wnp;
        wa.root_w = c->fr[wcur].w.as<double>();
        wa.root_wcap = c->fr[wcur].cap;
        wa.root_l = c->fr[wcur].l.as<double>();
        wa.root_level = L;
        wa.order = worder;
        wa.sol_u = sol_u;
        wa.head = &ctl->qhead;
        wa.tail = &ctl->qtail;
        wa.pending = &ctl->pending;
        wa.stack = c->stack.as<double>();
        wa.x_out = x_dev;
        wa.leaf_x = c->leaf_x.as<uint8_t>();
        wa.cap = cap;
        wa.n_found = &ctl->n_found;
        wa.counters = ctl->counters;
        wa.flags = ctl->flags;
        wa.t_first = &ctl->t_first;
        wa.t_start = &ctl->t_start;
        wa.deadline = p.time_cap_ms > 0 ? (unsigned long long)(p.time_cap_ms * c->wall_khz) : 0ull;
        wa.mode = mode;
        wa.bound = bound;
        wa.hfac = hfac;
        wa.rmax_d = (double)rmax;
        wa.rmax = rmax;
        wa.cvec = cvec;
        wa.budget = p.disc_budget;
        wa.disc_count = p.disc_count;
        wa.hoelder = p.hoelder;
        wa.onedir = p.onedir;
        MSP_TRY(hipEventRecord(c->ev[4], st));
        int grid = c->num_cus;
        if (small_tree && nleft == 0)
            grid = (int)std::min<int64_t>(c->num_cus, std::max<int64_t>(1, (2 * wnp + wblock - 1) / wblock));
        MSP_TRY(launch_walk(wa, dimp, wblock, grid, st));
        MSP_TRY(hipEventRecord(c->ev[5], st));
    } else {
        MSP_TRY(hipEventRecord(c->ev[4], st));
        MSP_TRY(hipEventRecord(c->ev[5], st));
    }
    Ctl h;
    MSP_TRY(hipMemcpyAsync(&h, ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    MSP_TRY(hipStreamSynchronize(st));

    *n_found = (int64_t)h.n_found;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->evals = (int64_t)h.counters[0];
        stats->nodes = (int64_t)h.counters[1];
        stats->expansions = (int64_t)h.counters[2];
        stats->leaves = (int64_t)h.counters[3];
        stats->roots = np0;
        stats->stages = stages;
        stats->root_level = L;
        stats->initial_items = ninit;
        stats->items = (int64_t)h.counters[4];
        stats->block = wblock;
        stats->split_depth = k - L0;
        stats->k = k;
        stats->gs_ms = elapsed(c->ev[0], c->ev[1]);
        stats->rootgen_ms = elapsed(c->ev[2], c->ev[3]);
        stats->kernel_ms = elapsed(c->ev[4], c->ev[5]);
        stats->ordering_ms = ordered ? elapsed(c->ev[6], c->ev[7]) : 0.0;
        stats->ttfs_ms =
            (h.t_first && h.t_start) ? (double)(h.t_first - h.t_start) / c->wall_khz + stats->ordering_ms : -1.0;
        stats->total_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_call).count();
    }
    if (h.flags[3]) return MSP_E_NUMERIC;
    if (h.flags[1]) return MSP_E_OVERFLOW;
    if (h.flags[2]) return MSP_E_TIMEOUT;
    if ((int64_t)h.n_found > cap) return MSP_E_CAPACITY;
    return MSP_OK;
}

// Limited discrepancy search for a first solution (paper, Section 3): walks
// with discrepancy budget B = 0, 1, 2, ... (each a first-solution walk that
// admits paths whose values' ranks in their levels' value orders sum to at
// most B), then one walk without a budget, which is exhaustive.  Stops at the first pass with a
// hit; counters and times are summed over the passes (stages = passes run).
static int lds_search(msp_ctx *c, int m, int n, const int32_t *A_dev, const int64_t *d_dev, const int64_t *basis_dev,
                      int k, int order, const msp_params *pin, uint8_t *x_dev, int64_t cap, int64_t *n_found,
                      msp_stats *stats, void *stream, const int64_t *cvec, long long rmax) {
    auto t0 = std::chrono::steady_clock::now();
    msp_params p;
    msp_params_default(&p);
    if (pin) p = *pin;
    if (!n_found) return MSP_E_ARG;
    if (p.root_begin != 0 || p.root_count >= 0) return MSP_E_ARG;  // root positions change from pass to pass
    msp_stats acc;
    std::memset(&acc, 0, sizeof(acc));
    acc.ttfs_ms = -1.0;
    int rc = MSP_OK, passes = 0;
    const int maxb = std::min(k, 255);
    for (int B = 0; B <= maxb + 1; ++B) {
        msp_params q = p;
        q.disc_budget = B <= maxb ? B : -1;
        // A budgeted tree is narrow, so reaching the first-solution root count
        // takes a deep split, and root generation is paid again on every pass.
        // Eight roots per walker keep that small; donation balances the walk.
        if (q.target_roots == 0) q.target_roots = 8 * 256 * c->num_cus;
        if (p.time_cap_ms > 0) {
            const double used =
                std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (used >= p.time_cap_ms) {
                rc = MSP_E_TIMEOUT;
                break;
            }
            q.time_cap_ms = p.time_cap_ms - used;
        }
        msp_stats st;
        std::memset(&st, 0, sizeof(st));
        const double before =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        rc = enumerate_impl(c, m, n, A_dev, d_dev, basis_dev, k, MSP_FIRST, order, &q, x_dev, cap, n_found, &st,
                            stream, nullptr, cvec, rmax, passes > 0);
        ++passes;
        acc.evals += st.evals;
        acc.nodes += st.nodes;
        acc.expansions += st.expansions;
        acc.leaves += st.leaves;
        acc.items += st.items;
        acc.roots = st.roots;
        acc.split_depth = st.split_depth;
        acc.k = st.k;
        acc.block = st.block;
        acc.root_level = st.root_level;
        acc.initial_items = st.initial_items;
        acc.gs_ms += st.gs_ms;
        acc.rootgen_ms += st.rootgen_ms;
        acc.ordering_ms += st.ordering_ms;
        acc.kernel_ms += st.kernel_ms;
        if (*n_found > 0) {  // also with MSP_E_CAPACITY or MSP_E_TIMEOUT: the rows are valid
            // host time of the earlier passes, then this pass up to its hit
            acc.ttfs_ms = before + (st.ttfs_ms >= 0.0 ? st.ttfs_ms + st.gs_ms + st.rootgen_ms : st.total_ms);
            break;
        }
        if (rc != MSP_OK) break;
        if (B > maxb) break;  // the unlimited walk found nothing: no solution
    }
    acc.stages = passes;
    acc.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = acc;
    return rc;
}

extern "C" {

int msp_enumerate(msp_ctx *c, int m, int n, const int32_t *A_dev, const int64_t *d_dev, const int64_t *basis_dev,
                  int k, int mode, int order, const msp_params *p, uint8_t *x_dev, int64_t cap, int64_t *n_found,
                  msp_stats *stats, void *stream) {
    if (mode == MSP_LDS)
        return lds_search(c, m, n, A_dev, d_dev, basis_dev, k, order, p, x_dev, cap, n_found, stats, stream, nullptr,
                          1);
    return enumerate_impl(c, m, n, A_dev, d_dev, basis_dev, k, mode, order, p, x_dev, cap, n_found, stats, stream);
}

namespace {
int lll_status(int32_t st) {
    switch (st) {
        case 0: return MSP_OK;
        case -2: return MSP_E_RANK;
        case -3: return MSP_E_NOT_ISOLATED;
        case -4: return MSP_E_OVERFLOW;
        default: return MSP_E_NUMERIC;
    }
}

// One launch reduces `cnt` instances; descriptors are copied to the device.
int run_lll(msp_ctx *c, std::vector<LllDesc> &h, const int32_t *A_dev, const int64_t *d_dev, int64_t *out,
            const msp_params &p, hipStream_t st, const int64_t *cvec = nullptr, long long rmax = 1) {
    const int cnt = (int)h.size();
    int maxn = 0;
    size_t work = 0;
    for (auto &e : h) {
        maxn = std::max(maxn, e.n);
        e.work_off = (int64_t)work;
        work += (size_t)(e.n + 1) * (e.m + e.n + 1);
    }
    MSP_TRY(c->lll_desc.ensure(sizeof(LllDesc) * cnt));
    MSP_TRY(c->lll_work.ensure(work * sizeof(long long)));
    LllDesc *dd = c->lll_desc.as<LllDesc>();
    MSP_TRY(hipMemcpyAsync(dd, h.data(), sizeof(LllDesc) * cnt, hipMemcpyHostToDevice, st));
    LllArgs la{};
    // the kernel reads every per-instance field through these strided views
    la.m = &dd->m;
    la.n = &dd->n;
    la.A = A_dev;
    la.A_off = &dd->A_off;
    la.d = d_dev;
    la.d_off = &dd->d_off;
    la.N = p.N;
    la.delta = p.delta;
    la.max_iters = 2000000;
    la.work = c->lll_work.as<long long>();
    la.work_off = &dd->work_off;
    la.out = out;
    la.out_off = &dd->out_off;
    la.status = &dd->status;
    la.kout = &dd->kout;
    la.iters = &dd->iters;
    la.stride = (int)(sizeof(LllDesc) / sizeof(int32_t));
    la.cvec = cvec;
    la.rmax = rmax;
    MSP_TRY(launch_lll(la, cnt, maxn, st));
    MSP_TRY(hipMemcpyAsync(h.data(), dd, sizeof(LllDesc) * cnt, hipMemcpyDeviceToHost, st));
    MSP_TRY(hipStreamSynchronize(st));
    return MSP_OK;
}
}  // namespace

// BKZ of `count` extracted kernel bases in place (each k x dim, basis i at
// basis_dev + i * bstride), one workgroup per basis in one launch; a basis
// whose entries would outgrow the exact Gram keeps its LLL form.
static int bkz_after_lll(msp_ctx *c, const msp_params &p, int64_t *basis_dev, int k, int dim, hipStream_t st,
                         int count = 1, int64_t bstride = 0) {
    if (p.bkz_block < 2 || k < 2 || count < 1) return MSP_OK;
    if (bkz_lds_bytes(k) > 160 * 1024) return MSP_E_UNSUPPORTED;
    if (count == 1) bstride = (int64_t)k * dim;
    const size_t nb = (size_t)k * dim * sizeof(int64_t);
    const size_t all = ((size_t)(count - 1) * bstride + (size_t)k * dim) * sizeof(int64_t);
    MSP_TRY(c->bkz_save.ensure(all));
    MSP_TRY(c->bkz_out.ensure((size_t)count * (2 * sizeof(int) + sizeof(long long))));
    MSP_TRY(hipMemcpyAsync(c->bkz_save.p, basis_dev, all, hipMemcpyDeviceToDevice, st));
    BkzArgs b{};
    b.k = k;
    b.dim = dim;
    b.B = basis_dev;
    b.bstride = bstride;
    b.count = count;
    b.beta = p.bkz_block;
    b.tours = p.bkz_tours > 0 ? p.bkz_tours : 1;
    b.delta = p.delta;
    b.max_nodes = 1ll << 18;
    b.max_lll_iters = 1ll << 16;
    b.nodes = c->bkz_out.as<long long>();
    b.out = reinterpret_cast<int *>(b.nodes + count);
    MSP_TRY(launch_bkz(b, st));
    std::vector<int> out((size_t)2 * count);
    MSP_TRY(hipMemcpyAsync(out.data(), b.out, sizeof(int) * out.size(), hipMemcpyDeviceToHost, st));
    MSP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < count; ++i) {
        if (out[2 * i] != -4) continue;  // entries too large for the exact Gram: keep the LLL basis
        MSP_TRY(hipMemcpyAsync(basis_dev + (size_t)i * bstride, c->bkz_save.as<int64_t>() + (size_t)i * bstride, nb,
                               hipMemcpyDeviceToDevice, st));
    }
    MSP_TRY(hipStreamSynchronize(st));
    return MSP_OK;
}

int msp_reduce(msp_ctx *c, int m, int n, const int32_t *A_dev, const int64_t *d_dev, const msp_params *pin,
               int64_t *basis_dev, int *k_out, void *stream) {
    if (!c || !A_dev || !d_dev || !basis_dev || !k_out) return MSP_E_ARG;
    if (m < 1 || n < 1 || m > n || n > MSP_MAX_N) return MSP_E_ARG;
    msp_params p;
    msp_params_default(&p);
    if (pin) p = *pin;
    if (p.N < 1 || !(p.delta > 0.25 && p.delta < 1.0)) return MSP_E_ARG;
    if (p.bkz_block < 0 || p.bkz_block == 1 || p.bkz_block > 40) return MSP_E_ARG;
    *k_out = 0;
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    std::vector<LllDesc> h(1);
    h[0] = LllDesc{m, n, 0, 0, 0, 0, 0, 0, 0};
    const int rc = run_lll(c, h, A_dev, d_dev, basis_dev, p, st);
    if (rc != MSP_OK) return rc;
    c->last_lll_iters = h[0].iters;
    const int s = lll_status(h[0].status);
    if (s != MSP_OK) return s;
    const int rb = bkz_after_lll(c, p, basis_dev, h[0].kout, n + 1, st);
    if (rb != MSP_OK) return rb;
    *k_out = h[0].kout;
    return MSP_OK;
}

// Shuffle of the n variables for copy r of msp_solve_first: identity for r = 0,
// else Fisher-Yates driven by splitmix64 of (seed, r).
static void restart_perm(uint32_t seed, int r, int n, int32_t *perm) {
    for (int j = 0; j < n; ++j) perm[j] = j;
    if (r == 0) return;
    uint64_t x = ((uint64_t)seed << 32) ^ (uint64_t)(uint32_t)r;
    auto next = [&x]() {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    for (int j = n - 1; j > 0; --j) {
        const int i = (int)(next() % (uint64_t)(j + 1));
        std::swap(perm[i], perm[j]);
    }
}

int msp_solve_first(msp_ctx *c, int m, int n, const int32_t *A_dev, const int64_t *d_dev, int order,
                    const msp_params *pin, uint8_t *x_dev, int64_t cap, int64_t *n_found, msp_stats *stats,
                    void *stream) {
    if (!c || !A_dev || !d_dev || !n_found || cap < 0 || (cap > 0 && !x_dev)) return MSP_E_ARG;
    if (m < 1 || n < 1 || m > n || n > MSP_MAX_N) return MSP_E_ARG;
    msp_params p;
    msp_params_default(&p);
    if (pin) p = *pin;
    if (p.restarts < 1 || p.restarts > 64) return MSP_E_ARG;
    if (p.root_begin != 0 || p.root_count >= 0) return MSP_E_ARG;
    if (p.N < 1 || !(p.delta > 0.25 && p.delta < 1.0)) return MSP_E_ARG;
    if (p.bkz_block < 0 || p.bkz_block == 1 || p.bkz_block > 40) return MSP_E_ARG;
    *n_found = 0;
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    auto ms_since = [](std::chrono::steady_clock::time_point a) {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - a).count();
    };
    const int R = p.restarts;
    const size_t mn = (size_t)m * n, bsz = (size_t)(n + 1) * (n + 1);
    // ---- the copies and their reduction, all at once ----
    std::vector<int32_t> perm((size_t)R * n);
    for (int r = 0; r < R; ++r) restart_perm(p.restart_seed, r, n, perm.data() + (size_t)r * n);
    MSP_TRY(c->rs_perm.ensure(perm.size() * sizeof(int32_t)));
    MSP_TRY(c->rs_A.ensure((size_t)R * mn * sizeof(int32_t)));
    MSP_TRY(c->rs_basis.ensure((size_t)R * bsz * sizeof(int64_t)));
    MSP_TRY(c->rs_x.ensure((size_t)std::max<int64_t>(cap, 1) * n));
    const int32_t *perm_dev = c->rs_perm.as<int32_t>();
    int32_t *A_cp = c->rs_A.as<int32_t>();
    int64_t *bases = c->rs_basis.as<int64_t>();
    MSP_TRY(hipMemcpyAsync(c->rs_perm.p, perm.data(), perm.size() * sizeof(int32_t), hipMemcpyHostToDevice, st));
    MSP_TRY(launch_permute_cols(A_dev, m, n, perm_dev, R, A_cp, st));
    std::vector<LllDesc> h(R);
    for (int r = 0; r < R; ++r) h[r] = LllDesc{m, n, (int64_t)(r * mn), 0, 0, (int64_t)(r * bsz), 0, 0, 0};
    int rc = run_lll(c, h, A_cp, d_dev, bases, p, st);
    if (rc != MSP_OK) return rc;
    const int s0 = lll_status(h[0].status);
    if (s0 != MSP_OK) return s0;
    const int k = h[0].kout;
    std::vector<char> ok(R);
    int nok = 0;
    for (int r = 0; r < R; ++r) nok += (ok[r] = lll_status(h[r].status) == MSP_OK && h[r].kout == k);
    if (nok == R) {
        rc = bkz_after_lll(c, p, bases, k, n + 1, st, R, (int64_t)bsz);
    } else {
        for (int r = 0; r < R && rc == MSP_OK; ++r)
            if (ok[r]) rc = bkz_after_lll(c, p, bases + (size_t)r * bsz, k, n + 1, st);
    }
    if (rc != MSP_OK) return rc;
    msp_stats acc;
    std::memset(&acc, 0, sizeof(acc));
    acc.reduce_ms = ms_since(t0);
    acc.ttfs_ms = -1.0;
    acc.copy = -1;
    acc.copies = nok;
    // ---- LDS passes in rounds: in round q copy r runs budget q - lag(r) ----
    // lag(r) = floor(log2(r + 1)): copy 0 leads, and each doubling of the
    // copy count trails by one budget.  A pass costs a few times the pass one
    // budget lower, so a round costs about two passes of copy 0 while every
    // copy still advances.  After every copy has run budget maxb, copy 0 runs
    // the unlimited, exhaustive pass.
    const auto ts = std::chrono::steady_clock::now();
    const int maxb = std::min(k, 255);
    auto lag = [](int r) {
        int l = 0;
        while ((2 << l) <= r + 1) ++l;
        return l;
    };
    const int last_round = maxb + lag(R - 1);
    int passes = 0;
    bool done = false;
    for (int round = 0; round <= last_round + 1 && !done; ++round) {
        for (int r = 0; r < R && !done; ++r) {
            if (!ok[r]) continue;
            int B = round - lag(r);
            if (round > last_round) {
                if (r > 0) break;  // the unlimited pass: copy 0 only, exhaustive
                B = maxb + 1;
            } else if (B < 0 || B > maxb) {
                continue;
            }
            msp_params q = p;
            q.disc_budget = B <= maxb ? B : -1;
            if (q.target_roots == 0) q.target_roots = 8 * 256 * c->num_cus;
            if (p.time_cap_ms > 0) {
                const double used = ms_since(ts);
                if (used >= p.time_cap_ms) {
                    rc = MSP_E_TIMEOUT;
                    done = true;
                    break;
                }
                q.time_cap_ms = p.time_cap_ms - used;
            }
            const double before = ms_since(t0);
            int64_t nf = 0;
            msp_stats sti;
            std::memset(&sti, 0, sizeof(sti));
            rc = enumerate_impl(c, m, n, A_cp + (size_t)r * mn, d_dev, bases + (size_t)r * bsz, k, MSP_FIRST, order,
                                &q, r == 0 ? x_dev : c->rs_x.as<uint8_t>(), cap, &nf, &sti, stream);
            ++passes;
            acc.evals += sti.evals;
            acc.nodes += sti.nodes;
            acc.expansions += sti.expansions;
            acc.leaves += sti.leaves;
            acc.items += sti.items;
            acc.roots = sti.roots;
            acc.split_depth = sti.split_depth;
            acc.k = sti.k;
            acc.block = sti.block;
            acc.root_level = sti.root_level;
            acc.initial_items = sti.initial_items;
            acc.gs_ms += sti.gs_ms;
            acc.rootgen_ms += sti.rootgen_ms;
            acc.ordering_ms += sti.ordering_ms;
            acc.kernel_ms += sti.kernel_ms;
            // a hit counts also when the pass ends with MSP_E_CAPACITY (more
            // hits than cap rows) or MSP_E_TIMEOUT: its rows are valid
            if (nf > 0) {
                if (r > 0 && cap > 0) {
                    MSP_TRY(launch_unpermute_rows(c->rs_x.as<uint8_t>(), std::min(nf, cap), n,
                                                  perm_dev + (size_t)r * n, x_dev, st));
                    MSP_TRY(hipStreamSynchronize(st));
                }
                *n_found = nf;
                acc.copy = r;
                acc.ttfs_ms =
                    before + (sti.ttfs_ms >= 0.0 ? sti.ttfs_ms + sti.gs_ms + sti.rootgen_ms : sti.total_ms);
                done = true;
            }
            if (rc != MSP_OK) done = true;
        }
    }
    acc.stages = passes;
    acc.total_ms = ms_since(t0);
    if (stats) *stats = acc;
    return rc;
}

// n bucket of the tuned-root table: instances whose n differs by less than 16
// share their tuned root count.
static int n_bucket(int n) { return (n + 15) / 16; }

static int tuned_roots(const msp_ctx *c, int mode, int m, int n) {
    for (const auto &e : c->tuned)
        if (e.arch == c->arch && e.mode == mode && e.m == m && e.nbucket == n_bucket(n)) return e.target_roots;
    return 0;
}

int msp_tune_lookup(msp_ctx *c, int mode, int m, int n, int *target_roots) {
    if (!c || !target_roots || m < 1 || n < 1) return MSP_E_ARG;
    *target_roots = tuned_roots(c, mode, m, n);
    return MSP_OK;
}

int msp_solve_batch(msp_ctx *c, int batch, const msp_batch_desc *desc, const int32_t *A_dev, const int64_t *d_dev,
                    int mode, int order, const msp_params *pin, uint8_t *x_dev, int64_t *n_found, int32_t *status,
                    msp_stats *stats, void *stream) {
    if (!c || batch < 1 || !desc || !A_dev || !d_dev || !n_found || !status) return MSP_E_ARG;
    for (int i = 0; i < batch; ++i) {
        const msp_batch_desc &e = desc[i];
        if (e.m < 1 || e.n < 1 || e.m > e.n || e.n > MSP_MAX_N || e.A_off < 0 || e.d_off < 0 || e.x_off < 0 ||
            e.cap < 0 || (e.cap > 0 && !x_dev))
            return MSP_E_ARG;
    }
    msp_params p;
    msp_params_default(&p);
    if (pin) p = *pin;
    if (p.N < 1 || !(p.delta > 0.25 && p.delta < 1.0)) return MSP_E_ARG;
    if (p.bkz_block < 0 || p.bkz_block == 1 || p.bkz_block > 40) return MSP_E_ARG;
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    auto t0 = std::chrono::steady_clock::now();
    // ---- steps 1-2 for the whole batch in one launch ----
    std::vector<LllDesc> h(batch);
    size_t boff = 0;
    for (int i = 0; i < batch; ++i) {
        h[i] = LllDesc{desc[i].m, desc[i].n, desc[i].A_off, desc[i].d_off, 0, (int64_t)boff, 0, 0, 0};
        boff += (size_t)(desc[i].n + 1) * (desc[i].n + 1);
    }
    MSP_TRY(c->batch_basis.ensure(boff * sizeof(int64_t)));
    int64_t *bases = c->batch_basis.as<int64_t>();
    int rc = run_lll(c, h, A_dev, d_dev, bases, p, st);
    if (rc != MSP_OK) return rc;
    // optional BKZ of each kernel basis (shapes differ, so one launch each)
    std::vector<int> bkz_rc(batch, MSP_OK);
    if (p.bkz_block >= 2)
        for (int i = 0; i < batch; ++i)
            if (lll_status(h[i].status) == MSP_OK)
                bkz_rc[i] = bkz_after_lll(c, p, bases + h[i].out_off, h[i].kout, desc[i].n + 1, st);
    const double reduce_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / batch;
    // ---- steps 3-4 per instance ----
    int first_bad = MSP_OK;
    for (int i = 0; i < batch; ++i) {
        const msp_batch_desc &e = desc[i];
        n_found[i] = 0;
        int s = lll_status(h[i].status);
        if (s == MSP_OK) s = bkz_rc[i];
        msp_stats sti;
        std::memset(&sti, 0, sizeof(sti));
        if (s == MSP_OK && mode == MSP_LDS)
            s = lds_search(c, e.m, e.n, A_dev + e.A_off, d_dev + e.d_off, bases + h[i].out_off, h[i].kout, order, &p,
                           x_dev ? x_dev + e.x_off : nullptr, e.cap, &n_found[i], &sti, stream, nullptr, 1);
        else if (s == MSP_OK) {
            // a root count tuned for this shape by msp_autotune, unless the caller set one
            msp_params q = p;
            if (q.target_roots == 0 && q.split_depth < 0) q.target_roots = tuned_roots(c, mode, e.m, e.n);
            s = enumerate_impl(c, e.m, e.n, A_dev + e.A_off, d_dev + e.d_off, bases + h[i].out_off, h[i].kout, mode,
                               order, &q, x_dev ? x_dev + e.x_off : nullptr, e.cap, &n_found[i], &sti, stream);
        }
        sti.reduce_ms = reduce_ms;
        status[i] = s;
        if (stats) stats[i] = sti;
        if (s != MSP_OK && first_bad == MSP_OK) first_bad = s;
    }
    return first_bad;
}


// r_max and c_j of the bounds r_dev (device), into the context; returns
// MSP_OK and *rmax_out, or MSP_E_ARG / MSP_E_OVERFLOW.
static int bounds_setup(msp_ctx *c, int n, const int32_t *r_dev, long long *rmax_out, hipStream_t st) {
    MSP_TRY(c->cvec.ensure((size_t)n * sizeof(int64_t)));
    MSP_TRY(c->rmax.ensure(sizeof(long long)));
    MSP_TRY(launch_bounds_scale(r_dev, n, c->cvec.as<int64_t>(), c->rmax.as<long long>(), st));
    long long rm = 0;
    MSP_TRY(hipMemcpyAsync(&rm, c->rmax.p, sizeof(rm), hipMemcpyDeviceToHost, st));
    MSP_TRY(hipStreamSynchronize(st));
    if (rm == -1) return MSP_E_ARG;
    if (rm < 1) return MSP_E_OVERFLOW;
    *rmax_out = rm;
    return MSP_OK;
}

int msp_reduce_bounded(msp_ctx *c, int m, int n, const int32_t *A_dev, const int64_t *d_dev, const int32_t *r_dev,
                       const msp_params *pin, int64_t *basis_dev, int *k_out, void *stream) {
    if (!c || !A_dev || !d_dev || !r_dev || !basis_dev || !k_out) return MSP_E_ARG;
    if (m < 1 || n < 1 || m > n || n > MSP_MAX_N) return MSP_E_ARG;
    msp_params p;
    msp_params_default(&p);
    if (pin) p = *pin;
    if (p.N < 1 || !(p.delta > 0.25 && p.delta < 1.0)) return MSP_E_ARG;
    if (p.bkz_block < 0 || p.bkz_block == 1 || p.bkz_block > 40) return MSP_E_ARG;
    *k_out = 0;
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    long long rmax = 1;
    int rc = bounds_setup(c, n, r_dev, &rmax, st);
    if (rc != MSP_OK) return rc;
    std::vector<LllDesc> h(1);
    h[0] = LllDesc{m, n, 0, 0, 0, 0, 0, 0, 0};
    rc = run_lll(c, h, A_dev, d_dev, basis_dev, p, st, c->cvec.as<int64_t>(), rmax);
    if (rc != MSP_OK) return rc;
    c->last_lll_iters = h[0].iters;
    const int s = lll_status(h[0].status);
    if (s != MSP_OK) return s;
    const int rb = bkz_after_lll(c, p, basis_dev, h[0].kout, n + 1, st);
    if (rb != MSP_OK) return rb;
    *k_out = h[0].kout;
    return MSP_OK;
}

int msp_enumerate_bounded(msp_ctx *c, int m, int n, const int32_t *A_dev, const int64_t *d_dev, const int32_t *r_dev,
                          const int64_t *basis_dev, int k, int mode, int order, const msp_params *p, uint8_t *x_dev,
                          int64_t cap, int64_t *n_found, msp_stats *stats, void *stream) {
    if (!c || !r_dev || n < 1 || n > MSP_MAX_N) return MSP_E_ARG;
    DeviceGuard g(c->device);
    long long rmax = 1;
    int rc = bounds_setup(c, n, r_dev, &rmax, (hipStream_t)stream);
    if (rc != MSP_OK) return rc;
    if (mode == MSP_LDS)
        return lds_search(c, m, n, A_dev, d_dev, basis_dev, k, order, p, x_dev, cap, n_found, stats, stream,
                          c->cvec.as<int64_t>(), rmax);
    return enumerate_impl(c, m, n, A_dev, d_dev, basis_dev, k, mode, order, p, x_dev, cap, n_found, stats, stream,
                          nullptr, c->cvec.as<int64_t>(), rmax);
}

int msp_solve_box(msp_ctx *c, int m, int n, const int32_t *A_dev, const int64_t *d_dev, const int32_t *lo_dev,
                  const int32_t *hi_dev, int mode, int order, const msp_params *p, int32_t *x_dev, int64_t cap,
                  int64_t *n_found, msp_stats *stats, void *stream) {
    if (!c || !A_dev || !d_dev || !lo_dev || !hi_dev || !n_found || cap < 0 || (cap > 0 && !x_dev)) return MSP_E_ARG;
    if (m < 1 || n < 1 || m > n || n > MSP_MAX_N) return MSP_E_ARG;
    *n_found = 0;
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    MSP_TRY(c->box_d.ensure((size_t)m * sizeof(int64_t)));
    MSP_TRY(c->box_r.ensure((size_t)n * sizeof(int32_t)));
    MSP_TRY(c->box_basis.ensure((size_t)(n + 1) * (n + 1) * sizeof(int64_t)));
    MSP_TRY(c->box_x.ensure((size_t)std::max<int64_t>(cap, 1) * n));
    MSP_TRY(c->box_st.ensure(sizeof(int)));
    // x := x - l, d := d - A l, r := u - l (Section 2)
    MSP_TRY(launch_box_setup(m, n, A_dev, d_dev, lo_dev, hi_dev, c->box_d.as<int64_t>(), c->box_r.as<int32_t>(),
                             c->box_st.as<int>(), st));
    int bad = 0;
    MSP_TRY(hipMemcpyAsync(&bad, c->box_st.p, sizeof(int), hipMemcpyDeviceToHost, st));
    MSP_TRY(hipStreamSynchronize(st));
    if (bad) return MSP_E_ARG;
    int k = 0;
    int rc = msp_reduce_bounded(c, m, n, A_dev, c->box_d.as<int64_t>(), c->box_r.as<int32_t>(), p,
                                c->box_basis.as<int64_t>(), &k, stream);
    if (rc != MSP_OK) return rc;
    rc = msp_enumerate_bounded(c, m, n, A_dev, c->box_d.as<int64_t>(), c->box_r.as<int32_t>(),
                               c->box_basis.as<int64_t>(), k, mode, order, p, c->box_x.as<uint8_t>(), cap, n_found,
                               stats, stream);
    if (rc != MSP_OK && rc != MSP_E_CAPACITY && rc != MSP_E_TIMEOUT) return rc;
    // x = x' + l for every row written
    MSP_TRY(launch_box_shift(std::min<int64_t>(*n_found, cap), n, c->box_x.as<uint8_t>(), lo_dev, x_dev, st));
    MSP_TRY(hipStreamSynchronize(st));
    return rc;
}

int msp_autotune(msp_ctx *c, int batch, const msp_batch_desc *desc, const int32_t *A_dev, const int64_t *d_dev,
                 int mode, int order, const msp_params *base, msp_params *best, msp_tune_point *points, int *npoints,
                 void *stream) {
    if (!c || batch < 1 || !desc || !A_dev || !d_dev || !best) return MSP_E_ARG;
    if (mode != MSP_ALL && mode != MSP_FIRST) return MSP_E_ARG;
    for (int i = 0; i < batch; ++i) {
        const msp_batch_desc &e = desc[i];
        if (e.m < 1 || e.n < 1 || e.m > e.n || e.n > MSP_MAX_N || e.A_off < 0 || e.d_off < 0) return MSP_E_ARG;
    }
    msp_params p;
    msp_params_default(&p);
    if (base) p = *base;
    if (p.N < 1 || !(p.delta > 0.25 && p.delta < 1.0)) return MSP_E_ARG;
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    std::vector<LllDesc> h(batch);
    size_t boff = 0;
    int maxn = 0;
    for (int i = 0; i < batch; ++i) {
        h[i] = LllDesc{desc[i].m, desc[i].n, desc[i].A_off, desc[i].d_off, 0, (int64_t)boff, 0, 0, 0};
        boff += (size_t)(desc[i].n + 1) * (desc[i].n + 1);
        maxn = std::max(maxn, desc[i].n);
    }
    MSP_TRY(c->batch_basis.ensure(boff * sizeof(int64_t)));
    int64_t *bases = c->batch_basis.as<int64_t>();
    int rc = run_lll(c, h, A_dev, d_dev, bases, p, st);
    if (rc != MSP_OK) return rc;
    for (int i = 0; i < batch; ++i)
        if (lll_status(h[i].status) != MSP_OK) return lll_status(h[i].status);
    const int per_cu_all[] = {128, 256, 512, 1024, 2048};
    const int per_cu_first[] = {4096, 16384, 65536};
    const int *cand = mode == MSP_ALL ? per_cu_all : per_cu_first;
    const int ncand = mode == MSP_ALL ? 5 : 3;
    // first-solution tuning needs an output row per instance; exhaustive
    // tuning counts only
    MSP_TRY(c->trace_x.ensure((size_t)64 * (maxn > 0 ? maxn : 1)));
    double best_ms = -1.0;
    int best_t = 0;
    // per shape group (m, n bucket): summed time and status of each candidate
    std::vector<std::pair<int, int>> groups;
    std::vector<int> gi(batch);
    for (int i = 0; i < batch; ++i) {
        const std::pair<int, int> key{desc[i].m, n_bucket(desc[i].n)};
        auto it = std::find(groups.begin(), groups.end(), key);
        gi[i] = (int)(it - groups.begin());
        if (it == groups.end()) groups.push_back(key);
    }
    std::vector<double> gms((size_t)ncand * groups.size(), 0.0);
    std::vector<int> gok((size_t)ncand * groups.size(), 1);
    for (int ci = 0; ci < ncand; ++ci) {
        msp_params q = p;
        q.target_roots = cand[ci] * c->num_cus;
        q.split_depth = -1;
        double tot = 0.0;
        int st_first = MSP_OK;
        for (int i = 0; i < batch; ++i) {
            const msp_batch_desc &e = desc[i];
            int64_t nf = 0;
            msp_stats sti;
            const int s = enumerate_impl(c, e.m, e.n, A_dev + e.A_off, d_dev + e.d_off, bases + h[i].out_off,
                                         h[i].kout, mode, order, &q, c->trace_x.as<uint8_t>(), 64, &nf, &sti, stream);
            if (s != MSP_OK && s != MSP_E_CAPACITY && st_first == MSP_OK) st_first = s;
            if (s != MSP_OK && s != MSP_E_CAPACITY && s != MSP_E_TIMEOUT) return s;
            const double ms = sti.rootgen_ms + sti.ordering_ms + sti.kernel_ms;
            tot += ms;
            gms[(size_t)ci * groups.size() + gi[i]] += ms;
            if (s != MSP_OK && s != MSP_E_CAPACITY) gok[(size_t)ci * groups.size() + gi[i]] = 0;
        }
        if (points && ci < 8) points[ci] = msp_tune_point{q.target_roots, st_first, tot};
        if (st_first == MSP_OK && (best_ms < 0.0 || tot < best_ms)) {
            best_ms = tot;
            best_t = q.target_roots;
        }
    }
    if (npoints) *npoints = ncand;
    if (best_ms < 0.0) return MSP_E_TIMEOUT;  // no candidate finished every instance
    // the fastest candidate of each shape group goes into the context's table
    for (size_t g2 = 0; g2 < groups.size(); ++g2) {
        int bt = 0;
        double bms = -1.0;
        for (int ci = 0; ci < ncand; ++ci) {
            const size_t ix = (size_t)ci * groups.size() + g2;
            if (gok[ix] && (bms < 0.0 || gms[ix] < bms)) {
                bms = gms[ix];
                bt = cand[ci] * c->num_cus;
            }
        }
        if (bt == 0) continue;
        bool found = false;
        for (auto &e : c->tuned)
            if (e.arch == c->arch && e.mode == mode && e.m == groups[g2].first && e.nbucket == groups[g2].second) {
                e.target_roots = bt;
                found = true;
            }
        if (!found) c->tuned.push_back({c->arch, mode, groups[g2].first, groups[g2].second, bt});
    }
    *best = p;
    best->target_roots = best_t;
    best->split_depth = -1;
    return MSP_OK;
}

// ---------------------------------------------------------------------------
// Root traces and the root-scoring model.

int msp_root_trace(msp_ctx *c, int m, int n, const int32_t *A_dev, const int64_t *d_dev, const int64_t *basis_dev,
                   int k, const msp_params *p, float *feat_dev, uint8_t *label_dev, int64_t cap_roots,
                   int64_t *nroots, int64_t *n_found, msp_stats *stats, void *stream) {
    if (!c || !nroots || !n_found || cap_roots < 0 || (cap_roots > 0 && (!feat_dev || !label_dev))) return MSP_E_ARG;
    *nroots = 0;
    *n_found = 0;
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t scap = kTraceSolutions;
    if (n < 1 || k < 1) return MSP_E_ARG;
    MSP_TRY(c->trace_x.ensure((size_t)scap * n));
    MSP_TRY(c->sol_u.ensure((size_t)scap * k));
    int rc = enumerate_impl(c, m, n, A_dev, d_dev, basis_dev, k, MSP_ALL, MSP_PLAIN, p, c->trace_x.as<uint8_t>(), scap,
                            n_found, stats, stream, c->sol_u.as<int8_t>());
    if (rc != MSP_OK) return rc;
    const int64_t np = c->last_np;
    *nroots = np;
    if (np > cap_roots) return MSP_E_CAPACITY;
    if (np == 0) return MSP_OK;
    FeatArgs fa{c->last_k, c->last_dim, c->last_m, c->last_L, c->last_ws, c->fr[c->last_cur].view(), np,
                c->gs_mu.as<double>(), c->gs_beta.as<double>(), c->last_R, feat_dev};
    MSP_TRY(launch_root_features(fa, st));
    MSP_TRY(launch_root_labels(c->fr[c->last_cur].view(), np, c->last_k, c->last_L, c->sol_u.as<int8_t>(),
                               std::min<int64_t>(*n_found, scap), label_dev, st));
    MSP_TRY(hipStreamSynchronize(st));
    return MSP_OK;
}

namespace {
int model_alloc(msp_ctx *c) {
    const size_t nb = (size_t)kNumParams * sizeof(float);
    MSP_TRY(c->w_master.ensure(nb));
    MSP_TRY(c->w_q.ensure(nb));
    MSP_TRY(c->adam_m.ensure(nb));
    MSP_TRY(c->adam_v.ensure(nb));
    MSP_TRY(c->step.ensure(sizeof(unsigned long long)));
    MSP_TRY(c->dev_loss.ensure(sizeof(float)));
    MSP_TRY(c->npos.ensure(sizeof(unsigned long long)));
    if (!c->aux) MSP_TRY(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
    return MSP_OK;
}

int model_upload(msp_ctx *c, const float *w) {
    int rc = model_alloc(c);
    if (rc != MSP_OK) return rc;
    hipStream_t st = c->aux;
    MSP_TRY(hipMemcpyAsync(c->w_master.p, w, (size_t)kNumParams * sizeof(float), hipMemcpyHostToDevice, st));
    MSP_TRY(launch_bf16_round(c->w_master.as<float>(), c->w_q.as<float>(), st));
    MSP_TRY(hipStreamSynchronize(st));
    c->has_model = true;
    return MSP_OK;
}
}  // namespace

int msp_model_init(msp_ctx *c, uint64_t seed) {
    if (!c) return MSP_E_ARG;
    DeviceGuard g(c->device);
    // He-normal weights for the ReLU layers, N(0, 1/64) for the output
    // layer, zero biases.
    std::vector<float> w(kNumParams, 0.0f);
    std::mt19937_64 rng(seed);
    std::normal_distribution<float> n1(0.0f, std::sqrt(2.0f / kNumFeat)), n2(0.0f, std::sqrt(2.0f / kHidden)),
        n3(0.0f, std::sqrt(1.0f / kHidden));
    size_t o = 0;
    for (int i = 0; i < kHidden * kNumFeat; ++i) w[o++] = n1(rng);
    o += kHidden;
    for (int i = 0; i < kHidden * kHidden; ++i) w[o++] = n2(rng);
    o += kHidden;
    for (int i = 0; i < kHidden; ++i) w[o++] = n3(rng);
    return model_upload(c, w.data());
}

int msp_model_set(msp_ctx *c, const float *w) {
    if (!c || !w) return MSP_E_ARG;
    for (int i = 0; i < kNumParams; ++i)
        if (!std::isfinite(w[i])) return MSP_E_ARG;
    DeviceGuard g(c->device);
    return model_upload(c, w);
}

int msp_model_get(msp_ctx *c, float *w) {
    if (!c || !w || !c->has_model) return MSP_E_ARG;
    DeviceGuard g(c->device);
    MSP_TRY(hipMemcpyAsync(w, c->w_master.p, (size_t)kNumParams * sizeof(float), hipMemcpyDeviceToHost, c->aux));
    MSP_TRY(hipStreamSynchronize(c->aux));
    return MSP_OK;
}

int msp_model_score(msp_ctx *c, const float *feat_dev, int64_t count, float *logit_dev, void *stream) {
    if (!c || count < 0 || (count > 0 && (!feat_dev || !logit_dev)) || !c->has_model) return MSP_E_ARG;
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    MSP_TRY(launch_mlp_score(c->w_q.as<float>(), feat_dev, count, logit_dev, st));
    MSP_TRY(hipStreamSynchronize(st));
    return MSP_OK;
}

int msp_model_grad(msp_ctx *c, const float *feat_dev, const uint8_t *label_dev, int64_t count, float pos_weight,
                   float *grad_dev, float *loss, void *stream) {
    if (!c || count < 1 || !feat_dev || !label_dev || !grad_dev || !loss || !c->has_model) return MSP_E_ARG;
    if (!(pos_weight > 0.0f) || count > (int64_t)INT32_MAX) return MSP_E_ARG;
    DeviceGuard g(c->device);
    hipStream_t st = (hipStream_t)stream;
    const int64_t waves = (count + 63) / 64;
    if (waves > (int64_t)INT32_MAX) return MSP_E_ARG;
    MSP_TRY(c->partial.ensure((size_t)waves * kPartialStride * sizeof(float)));
    MlpGradArgs ga{c->w_q.as<float>(), feat_dev, label_dev, nullptr, count, count, nullptr, 1, pos_weight,
                   c->partial.as<float>()};
    MSP_TRY(launch_mlp_grad(ga, (int)waves, st));
    MSP_TRY(launch_grad_sum(c->partial.as<float>(), (int)waves, grad_dev, c->dev_loss.as<float>(), st));
    MSP_TRY(hipMemcpyAsync(loss, c->dev_loss.p, sizeof(float), hipMemcpyDeviceToHost, st));
    MSP_TRY(hipStreamSynchronize(st));
    return MSP_OK;
}

int msp_train_params_default(msp_train_params *tp) {
    if (!tp) return MSP_E_ARG;
    tp->epochs = 20;
    tp->batch = 8192;
    tp->lr = 1e-3f;
    tp->pos_weight = 0.0f;
    tp->seed = 1;
    tp->use_graph = 1;
    return MSP_OK;
}

int msp_model_train(msp_ctx *c, const float *feat_dev, const uint8_t *label_dev, int64_t count,
                    const msp_train_params *tpin, float *loss_per_epoch, void *stream) {
    if (!c || count < 1 || !feat_dev || !label_dev || !c->has_model) return MSP_E_ARG;
    msp_train_params tp;
    msp_train_params_default(&tp);
    if (tpin) tp = *tpin;
    if (tp.epochs < 1 || tp.batch < 64 || tp.batch % 64 != 0 || !(tp.lr > 0.0f) || count > (int64_t)INT32_MAX)
        return MSP_E_ARG;
    DeviceGuard g(c->device);
    hipStream_t caller = (hipStream_t)stream;
    MSP_TRY(hipStreamSynchronize(caller));  // inputs were produced on the caller's stream
    hipStream_t st = c->aux;
    const int64_t B = tp.batch;
    const int64_t spe = (count + B - 1) / B;
    const int waves = (int)(B / 64);
    MSP_TRY(c->partial.ensure((size_t)waves * kPartialStride * sizeof(float)));
    MSP_TRY(c->loss_acc.ensure((size_t)tp.epochs * sizeof(float)));
    MSP_TRY(c->sh_keys.ensure((size_t)count * sizeof(uint32_t)));
    MSP_TRY(c->sh_keys_out.ensure((size_t)count * sizeof(uint32_t)));
    MSP_TRY(c->sh_idx.ensure((size_t)count * sizeof(int32_t)));
    MSP_TRY(c->sh_perm.ensure((size_t)count * sizeof(int32_t)));
    size_t tb = 0;
    MSP_TRY(shuffle_perm(nullptr, &tb, c->sh_keys.as<uint32_t>(), c->sh_keys_out.as<uint32_t>(),
                         c->sh_idx.as<int32_t>(), c->sh_perm.as<int32_t>(), count, tp.seed, 0, st));
    MSP_TRY(c->sh_tmp.ensure(tb));
    float pw = tp.pos_weight;
    if (!(pw > 0.0f)) {
        // balance the classes: weight positives by negatives / positives
        MSP_TRY(hipMemsetAsync(c->npos.p, 0, sizeof(unsigned long long), st));
        MSP_TRY(launch_count_pos(label_dev, count, c->npos.as<unsigned long long>(), st));
        unsigned long long npos = 0;
        MSP_TRY(hipMemcpyAsync(&npos, c->npos.p, sizeof(npos), hipMemcpyDeviceToHost, st));
        MSP_TRY(hipStreamSynchronize(st));
        pw = npos > 0 ? (float)((double)(count - (int64_t)npos) / (double)npos) : 1.0f;
        if (pw < 1.0f) pw = 1.0f;
    }
    // fresh optimizer state
    MSP_TRY(hipMemsetAsync(c->adam_m.p, 0, (size_t)kNumParams * sizeof(float), st));
    MSP_TRY(hipMemsetAsync(c->adam_v.p, 0, (size_t)kNumParams * sizeof(float), st));
    MSP_TRY(hipMemsetAsync(c->step.p, 0, sizeof(unsigned long long), st));
    MSP_TRY(hipMemsetAsync(c->loss_acc.p, 0, (size_t)tp.epochs * sizeof(float), st));
    MlpGradArgs ga{c->w_q.as<float>(), feat_dev, label_dev, c->sh_perm.as<int32_t>(), count, B,
                   c->step.as<unsigned long long>(), spe, pw, c->partial.as<float>()};
    AdamArgs aa{c->w_master.as<float>(), c->w_q.as<float>(), c->adam_m.as<float>(), c->adam_v.as<float>(),
                c->partial.as<float>(), waves, c->step.as<unsigned long long>(), spe, tp.lr,
                c->loss_acc.as<float>()};
    // One epoch = spe optimizer steps; every kernel reads the step counter
    // from device memory, so the same launches (or their graph) replay for
    // every epoch.
    hipGraphExec_t exec = nullptr;
    if (tp.use_graph) {
        hipGraph_t graph = nullptr;
        MSP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int64_t s = 0; s < spe && e == hipSuccess; ++s) {
            e = launch_mlp_grad(ga, waves, st);
            if (e == hipSuccess) e = launch_adam(aa, st);
        }
        hipError_t e2 = hipStreamEndCapture(st, &graph);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return map_err(e != hipSuccess ? e : e2);
        }
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) return map_err(e);
    }
    int rc = MSP_OK;
    for (int ep = 0; ep < tp.epochs && rc == MSP_OK; ++ep) {
        size_t tbe = c->sh_tmp.cap;
        hipError_t e = shuffle_perm(c->sh_tmp.p, &tbe, c->sh_keys.as<uint32_t>(), c->sh_keys_out.as<uint32_t>(),
                                    c->sh_idx.as<int32_t>(), c->sh_perm.as<int32_t>(), count, tp.seed, ep, st);
        if (e == hipSuccess) {
            if (exec) {
                e = hipGraphLaunch(exec, st);
            } else {
                for (int64_t s = 0; s < spe && e == hipSuccess; ++s) {
                    e = launch_mlp_grad(ga, waves, st);
                    if (e == hipSuccess) e = launch_adam(aa, st);
                }
            }
        }
        if (e != hipSuccess) rc = map_err(e);
    }
    if (rc == MSP_OK && loss_per_epoch) {
        hipError_t e = hipMemcpyAsync(loss_per_epoch, c->loss_acc.p, (size_t)tp.epochs * sizeof(float),
                                      hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) rc = map_err(e);
    }
    hipError_t e = hipStreamSynchronize(st);
    if (rc == MSP_OK && e != hipSuccess) rc = map_err(e);
    if (exec) (void)hipGraphExecDestroy(exec);
    return rc;
}

}  // extern "C"
