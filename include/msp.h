/*
 * msp.h -- C ABI of libmsp, a GPU (gfx950) solver for the market split
 * feasibility problem by lattice enumeration.
 *
 * Problem (paper, Section 1): given A in Z^{m x n} and d in Z^m (entries of
 * either sign, Section 2), find x in {0,1}^n with A x = d.  The method (Section 2):
 *   1. embed the problem in the lattice spanned by the n+1 columns of the
 *      (m+n+1) x (n+1) matrix of eq. (2), binary case r_max = c_i = 1,
 *      with a scale constant N (default 2^10);
 *   2. LLL-reduce that basis (step 1 of Algorithm 1) and keep the n-m+1
 *      reduced vectors whose first m entries vanish, dropping those entries
 *      (step 2) -- a basis b_0..b_{n-m} of the kernel lattice in Z^{n+1};
 *   3. Gram-Schmidt orthogonalise it (eq. (4), step 3);
 *   4. enumerate depth first every lattice vector v with ||v||_2^2 <= n+1
 *      that passes the Hoelder test of Thm 2 (Algorithm 1), and read the
 *      solutions off the vectors with ||v||_inf <= 1 (Thm 1).
 *
 * Conventions shared by every call:
 *   - Matrices are row-major.  A is int32 m x n; d is int64 m.
 *   - A kernel basis is int64 k x (n+1), k = n - m + 1, one basis vector per
 *     row; columns 0..n-1 are the variable coordinates (v_j = 2 x_j - 1 on
 *     a solution) and column n is the r_max coordinate (|v_n| = 1 on a
 *     solution).
 *   - Pointers named *_dev are device pointers on the context's device;
 *     all other pointers are host pointers.  The caller allocates and frees
 *     every buffer it passes.  The library never frees caller memory and
 *     keeps no caller pointer after a call returns: every call synchronises
 *     `stream` before returning.
 *   - `stream` is a hipStream_t (NULL = the null stream).
 *   - Every call returns MSP_OK (0) or a negative MSP_E_* code and never
 *     aborts or throws across the ABI.  msp_strerror() names a code.
 *   - A context is not thread safe: use one context per host thread.
 */
#ifndef MSP_H
#define MSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
enum {
    MSP_OK = 0,
    MSP_E_ARG = -1,          /* bad shape, null pointer, m > n, n > MSP_MAX_N     */
    MSP_E_RANK = -2,         /* more than n-m+1 zero-top vectors: rank A < m       */
    MSP_E_NOT_ISOLATED = -3, /* fewer than n-m+1 zero-top vectors: N too small,
                                the reduced basis does not split (Sec. 2)         */
    MSP_E_OVERFLOW = -4,     /* an integer bound was exceeded (see each call)      */
    MSP_E_CAPACITY = -5,     /* more solutions than `cap`; *n_found = true total   */
    MSP_E_TIMEOUT = -6,      /* time cap hit; partial results are valid            */
    MSP_E_DEVICE = -7,       /* a HIP runtime error                                */
    MSP_E_NOMEM = -8,        /* device allocation failed                           */
    MSP_E_UNSUPPORTED = -9,  /* shape outside the compiled kernel variants         */
    MSP_E_NUMERIC = -10      /* floating-point breakdown (non-positive GS norm)    */
};

#define MSP_MAX_N 127        /* largest n accepted (n + 1 <= 128)                */

/* Discrepancies (limited discrepancy search, Section 3).  Each level tries its
 * values in a fixed order: u1, u1+s, u1-s, u1+2s, ... around the centre, or
 * 0, 1, 2, ... while every higher value is zero.  Taking the value of rank r in
 * that order costs r discrepancies, and a path's discrepancies are the sum
 * over its levels.
 *
 * enumeration modes: every solution; a first solution by one walk; a first
 * solution by limited discrepancy search: walks that admit paths of at most
 * B = 0, 1, 2, ..., min(k, 255) discrepancies, then one walk without a budget
 * (exhaustive), stopping at the first pass with a hit.  msp_stats then sums
 * the passes (stages = passes run). */
enum { MSP_ALL = 0, MSP_FIRST = 1, MSP_LDS = 2 };
/* Orders in which the subtree roots are walked.  The order changes only
 * which solutions MSP_FIRST meets first and how soon; MSP_ALL returns the same
 * set and the same search-tree counters in every order.
 *   MSP_PLAIN        depth-first order (the order of Algorithm 1)
 *   MSP_LEARNED      best score first under the context's root-scoring model
 *                    (msp_model_init / msp_model_set / msp_model_train)
 *   MSP_DISCREPANCY  fewest discrepancies on the root's prefix first, then
 *                    depth-first: limited discrepancy search (Section 3)
 *                    applied to the roots */
enum { MSP_PLAIN = 0, MSP_LEARNED = 1, MSP_DISCREPANCY = 2 };

/* Root-scoring model: features per root and parameters of the MLP
 * 16 -> 64 -> 64 -> 1 (ReLU), used with BF16-rounded weights and FP32
 * accumulation.  Parameter vector layout (floats):
 *   W1[64][16] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3. */
#define MSP_NFEAT 16
#define MSP_MODEL_NPARAM 5313

typedef struct msp_ctx msp_ctx;

/* Tunables.  msp_params_default() fills the defaults given in brackets. */
typedef struct {
    int64_t N;            /* scale constant of eq. (2)                       [1024] */
    double delta;         /* LLL Lovász parameter                            [0.99] */
    double eps;           /* relative slack of both pruning tests            [1e-9] */
    int split_depth;      /* levels enumerated before the subtree split; -1 = auto [-1] */
    int block;            /* walk kernel workgroup size cap (256|512); 0 = auto [0] */
    int target_roots;     /* root count the automatic split aims for; 0 = auto:
                           * 512 per CU for MSP_ALL, 16384 per CU for MSP_FIRST,
                           * 2048 per CU for each MSP_LDS pass                 [0] */
    int hoelder;          /* 1: apply the Hoelder test (Thm 2)                  [1] */
    int onedir;           /* 1: apply the one-direction cut (Section 2)         [1] */
    double time_cap_ms;   /* enumeration wall-time cap; <= 0 = none             [0] */
    int refine;           /* MSP_FIRST with a non-plain order: refinement stages
                           * (see msp_enumerate); -1 = up to 64, 0 = off          [0] */
    int refine_keep;      /* best nodes expanded further per stage; 0 = auto
                           * (256 per CU)                                        [0] */
    int disc_budget;      /* at most this many discrepancies on any walked path
                           * (see above; Section 3); -1 = no limit, at most 255 [-1] */
    int bkz_block;        /* msp_reduce: BKZ block size applied to the kernel
                           * basis after LLL (Section 2); 0 = LLL only, else 2..40 [0] */
    int bkz_tours;        /* BKZ tour limit                                      [4] */
    int restarts;         /* msp_solve_first: shuffled copies of the instance,
                           * 1..64 (copy 0 keeps the given variable order)       [1] */
    uint32_t restart_seed;/* msp_solve_first: seed of the shuffles               [1] */
    int disc_count;       /* reading of a discrepancy (Section 3): 0 = a value's
                           * rank in its level's value order, 1 = one for every
                           * value other than the level's first              [0] */
    int64_t root_begin;   /* MSP_ALL / MSP_FIRST: walk only the subtree roots at
                           * positions root_begin .. root_begin + root_count - 1
                           * of the walk order (depth-first, or the root order's
                           * ranking), clipped to the roots there are.  Subtrees
                           * are independent, so the solution sets of disjoint
                           * ranges are disjoint, their union over a cover of the
                           * roots is the full set, and their counters add up to
                           * the full walk's (the levels above the split are
                           * counted by the call whose range starts at 0 only):
                           * a caller can checkpoint at a root
                           * position and resume there, or split the roots over
                           * several devices.  The split must be the same in
                           * every call (split_depth >= 0, or the same automatic
                           * split: same instance, basis and parameters).  Not
                           * with MSP_LDS or refinement (MSP_E_ARG).            [0] */
    int64_t root_count;   /* roots in the range; -1 = all from root_begin        [-1] */
} msp_params;

/* Counters and timings of one call (all times in milliseconds).
 * eval = a candidate u_t whose partial norm was computed; node = a candidate
 * that passed the l2 test; expansion = a node that passed the Hoelder test and
 * was descended into; leaf = a node at level 0. */
typedef struct {
    int64_t evals, nodes, expansions, leaves;
    int64_t roots;           /* subtree roots from root generation               */
    int64_t items;           /* work items walked (roots plus split-off items)   */
    int32_t split_depth;     /* split depth used                                 */
    int32_t k;               /* kernel lattice rank n - m + 1                    */
    int32_t block;           /* threads per workgroup of the walk kernel         */
    int32_t pad;
    double reduce_ms;        /* msp_reduce (embedding + LLL + extraction)        */
    double gs_ms;            /* Gram-Schmidt kernel                              */
    double rootgen_ms;       /* root generation (levels above the split)         */
    double ordering_ms;      /* root features, scores and sort (non-plain orders) */
    double kernel_ms;        /* walk kernel                                      */
    double ttfs_ms;          /* MSP_FIRST: ordering_ms + walk-kernel start to the
                              * first verified hit (device clock); -1 if none   */
    double total_ms;         /* whole call                                       */
    int32_t stages;          /* refinement stages run (0 without refinement)     */
    int32_t root_level;      /* level of the walked roots (deepest stage)        */
    int64_t initial_items;   /* work items before the walk: roots + leftovers    */
    int32_t copy;            /* msp_solve_first: the copy that hit (-1: none)    */
    int32_t copies;          /* msp_solve_first: copies reduced and searched     */
} msp_stats;

/* Fill `p` with the defaults.  Returns MSP_OK or MSP_E_ARG (p == NULL). */
int msp_params_default(msp_params *p);

/* Create a context bound to HIP device `device`.  The context owns its
 * workspace (root queue, walker stacks, counters, model weights), grown on
 * demand and freed by msp_ctx_destroy. */
int msp_ctx_create(int device, msp_ctx **out);
void msp_ctx_destroy(msp_ctx *ctx);

/* Steps 1-2 of Algorithm 1 on the GPU (Section 2, eq. (2)).
 * With p->bkz_block >= 2 the extracted kernel basis is further BKZ-reduced
 * with that block size (exact unimodular integer updates; the solution set
 * does not change, the enumeration tree usually shrinks); if an entry would
 * exceed 2^26 the LLL basis is returned instead.
 * Builds the embedding basis with scale p->N, LLL-reduces it in FP64 with
 * exact int64 basis updates (Lovász p->delta), keeps the reduced vectors whose
 * first m entries are zero and writes them, top entries dropped, to
 * basis_dev (int64 k x (n+1), capacity (n+1) x (n+1)); *k_out = k = n-m+1.
 * Errors: MSP_E_ARG, MSP_E_NOT_ISOLATED (other than k zero-top vectors),
 * MSP_E_OVERFLOW (an int64 entry or Gram entry beyond 2^53),
 * MSP_E_NUMERIC (LLL failed to converge), MSP_E_DEVICE. */
int msp_reduce(msp_ctx *ctx, int m, int n, const int32_t *A_dev, const int64_t *d_dev,
               const msp_params *p, int64_t *basis_dev, int *k_out, void *stream);

/* msp_reduce without any device allocation, for callers that cannot allocate
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It needs no context: it works on the calling thread's current
 * device, and `stream` must belong to that device.  Arguments, layouts and
 * results are those of msp_reduce with LLL only (p->bkz_block must be 0, or
 * MSP_E_ARG); k is returned in *k_out after the stream is synchronised.
 * Scratch: a file-scope device array of 261,376 bytes per GPU (a launch
 * descriptor and the (n+1) x (m+n+1) int64 embedding workspace, enough for
 * every n <= MSP_MAX_N), held until the process ends; a size beyond it is
 * rejected with MSP_E_ARG.  Calls that overlap on one GPU share the array and
 * race; serialise them. */
int msp_reduce_noalloc(int m, int n, const int32_t *A_dev, const int64_t *d_dev, const msp_params *p,
                       int64_t *basis_dev, int *k_out, void *stream);

/* Step 3 of Algorithm 1 (eq. (4)): FP64 Gram-Schmidt of a kernel basis.
 * basis_dev: int64 k x dim.  Outputs (device, caller-allocated):
 * bhat_dev k x dim (row i = b_hat_i), mu_dev k x k (mu_dev[i*k+j] = mu_ij for
 * j < i, 1 on the diagonal, 0 above), beta_dev k (||b_hat_i||^2).
 * Errors: MSP_E_ARG, MSP_E_NUMERIC (some beta_i <= 0: dependent basis). */
int msp_gram_schmidt(msp_ctx *ctx, int k, int dim, const int64_t *basis_dev,
                     double *bhat_dev, double *mu_dev, double *beta_dev, void *stream);

/* Step 3-4 of Algorithm 1 on a given kernel basis: Gram-Schmidt, root
 * generation above the split depth, and the subtree walk (Algorithm 1 with
 * the zig-zag order of next(), the l2 bound R = n+1, the Hoelder test and the
 * one-direction cut), with an exact check of every level-0 node (Thm 1, then
 * A x = d in integers).
 * mode MSP_ALL returns every solution exactly once (unspecified order);
 * MSP_FIRST stops at the first verified solution (one or a few rows).
 * order: MSP_PLAIN, MSP_LEARNED (needs a model: MSP_E_ARG otherwise) or
 * MSP_DISCREPANCY; see above.  With MSP_FIRST and a non-plain order the roots
 * are refined best first: the frontier is ordered, its best p->refine_keep
 * nodes are expanded a few more levels (in depth-first order) and ordered
 * again, stage after stage, until the frontier is deep; the walk then takes
 * the last frontier in order, followed by every stage's remaining nodes
 * (latest stage first, each in order).  The subtrees still cover the whole
 * tree once, so the result is as exhaustive as the plain walk.
 * x_dev: uint8 cap x n, rows of 0/1.  *n_found: solutions found (may exceed
 * cap: then only cap rows are written and MSP_E_CAPACITY is returned after the
 * full enumeration).  stats may be NULL.
 * Errors: MSP_E_ARG, MSP_E_UNSUPPORTED, MSP_E_OVERFLOW (|u_t| > 127 reached),
 * MSP_E_CAPACITY, MSP_E_TIMEOUT, MSP_E_NOMEM, MSP_E_DEVICE. */
int msp_enumerate(msp_ctx *ctx, int m, int n, const int32_t *A_dev, const int64_t *d_dev,
                  const int64_t *basis_dev, int k, int mode, int order, const msp_params *p,
                  uint8_t *x_dev, int64_t cap, int64_t *n_found, msp_stats *stats, void *stream);

/* Bounded variables (Section 2, eq. (2) in its general form): find x with
 * A x = d and 0 <= x_j <= r_j (a lower bound l is moved to 0 by the caller:
 * x := x - l, d := d - A l, r := r - l).  r_dev: int32 n, each 1..255
 * (MSP_E_ARG otherwise).  The library forms r_max = lcm(r_j) (MSP_E_OVERFLOW
 * beyond 2^20) and c_j = r_max / r_j; the embedding has -r_max / r_max in
 * vector 0 and 2 c_j on the diagonal; the enumeration bound is
 * R = (n+1) r_max^2, the Hoelder test is l > r_max ||w||_1 (1+eps), and a
 * leaf is a solution when v_n = +-r_max and |v_j| <= r_max (Thm 1), with
 * x_j = (v_j + r_max) / (2 c_j) written as uint8.  Otherwise as msp_reduce
 * and msp_enumerate (all r_j = 1 is the binary problem). */
int msp_reduce_bounded(msp_ctx *ctx, int m, int n, const int32_t *A_dev, const int64_t *d_dev,
                       const int32_t *r_dev, const msp_params *p, int64_t *basis_dev, int *k_out,
                       void *stream);
int msp_enumerate_bounded(msp_ctx *ctx, int m, int n, const int32_t *A_dev, const int64_t *d_dev,
                          const int32_t *r_dev, const int64_t *basis_dev, int k, int mode, int order,
                          const msp_params *p, uint8_t *x_dev, int64_t cap, int64_t *n_found,
                          msp_stats *stats, void *stream);

/* General box bounds l_j <= x_j <= u_j (Section 2): the library applies the
 * paper's substitution x := x - l, d := d - A l, r := u - l in a kernel, runs
 * msp_reduce_bounded and msp_enumerate_bounded on the shifted problem, and
 * writes x = x' + l.  lo_dev, hi_dev: int32 n with 1 <= u_j - l_j <= 255 and
 * |l_j|, |u_j| <= 2^24 (MSP_E_ARG otherwise).  x_dev: int32 cap x n, rows in
 * unspecified order.  Modes, orders, n_found, stats and errors as
 * msp_enumerate; the reduction (with p->bkz_block) is part of the call. */
int msp_solve_box(msp_ctx *ctx, int m, int n, const int32_t *A_dev, const int64_t *d_dev,
                  const int32_t *lo_dev, const int32_t *hi_dev, int mode, int order, const msp_params *p,
                  int32_t *x_dev, int64_t cap, int64_t *n_found, msp_stats *stats, void *stream);

/* One instance of a batch: A_dev + A_off holds its m x n matrix, d_dev +
 * d_off its right-hand side, x_dev + x_off its output rows (cap x n). */
typedef struct {
    int32_t m, n;
    int64_t A_off, d_off, x_off, cap;
} msp_batch_desc;

/* Reduce and enumerate a batch of independent instances of uneven shape
 * (Sections 1-2): one LLL launch reduces every instance (one wave each); with
 * p->bkz_block >= 2 each kernel basis is then BKZ-reduced as by msp_reduce;
 * then each instance is enumerated as by msp_enumerate on its own basis.
 * desc: host array of `batch` descriptors (offsets in elements).  Outputs
 * (host arrays of length batch): n_found[i], status[i] (an MSP_* code per
 * instance), stats[i] (may be NULL).  Returns MSP_OK when every instance
 * returned MSP_OK, otherwise the first non-OK instance status. */
int msp_solve_batch(msp_ctx *ctx, int batch, const msp_batch_desc *desc, const int32_t *A_dev,
                    const int64_t *d_dev, int mode, int order, const msp_params *p, uint8_t *x_dev,
                    int64_t *n_found, int32_t *status, msp_stats *stats, void *stream);

/* A first binary solution from A and d alone, by limited discrepancy search
 * over randomly shuffled copies of the instance (Section 4 proposes running the
 * method on randomly reordered input bases at once; here the copies share one
 * GPU).  Copy 0 is the instance as given; copy i > 0 permutes the variables by
 * a shuffle drawn from p->restart_seed and i.  All p->restarts copies are
 * reduced together (one LLL launch, then one BKZ launch when p->bkz_block >= 2,
 * one wave per copy).  The LDS passes (each as by msp_enumerate with MSP_LDS,
 * in `order`) then run in rounds q = 0, 1, 2, ...: in round q copy r runs
 * budget q - floor(log2(r + 1)), copies in index order, so copy 0 leads and
 * each doubling of the copy count trails by one budget.  The search stops at
 * the first verified hit.  Once every copy has run budget min(k, 255), copy 0
 * runs the unlimited pass, which is exhaustive.
 * x_dev receives up to `cap` rows in the caller's variable order, *n_found
 * their count (0 only if the instance has no solution, or on MSP_E_TIMEOUT).
 * stats holds the summed counters with copy and copies set; its reduce_ms is
 * the reduction of all copies, and its ttfs_ms runs from the start of the call
 * to the first verified hit (reduction included).  A copy whose reduction
 * fails (e.g. MSP_E_NOT_ISOLATED) is skipped; the call fails with that status
 * only if copy 0 fails.  p->time_cap_ms bounds the search after the
 * reduction.
 * Errors: those of msp_reduce and msp_enumerate; MSP_E_ARG for restarts
 * outside 1..64. */
int msp_solve_first(msp_ctx *ctx, int m, int n, const int32_t *A_dev, const int64_t *d_dev, int order,
                    const msp_params *p, uint8_t *x_dev, int64_t cap, int64_t *n_found, msp_stats *stats,
                    void *stream);

/* Autotuner (a project addition).  Reduces the `batch` tuning instances once
 * (as msp_solve_batch does), then for each candidate root count -- 128, 256,
 * 512, 1024 and 2048 roots per CU for MSP_ALL; 4096, 16384 and 65536 per CU
 * for MSP_FIRST -- enumerates every instance with *base and target_roots set
 * to the candidate, and times the enumeration (root generation, ordering and
 * walk; device events).  *best = *base with the fastest candidate's
 * target_roots.  points (may be NULL, room for 8) receives each candidate's
 * target_roots and total milliseconds; *npoints their count.  The result set
 * never depends on the candidate; only time does.
 * The context also keeps, per shape group of the tuning batch (m and the n
 * bucket ceil(n / 16)), the candidate fastest on that group, keyed by the
 * device architecture, the mode, m and the n bucket (a later call replaces
 * an entry).  msp_solve_batch then uses the tuned root count for every
 * instance of a tuned shape when p->target_roots == 0 and p->split_depth < 0
 * (modes MSP_ALL and MSP_FIRST). */
typedef struct {
    int32_t target_roots;
    int32_t status;          /* first non-OK status over the batch, or MSP_OK */
    double ms;               /* summed enumeration time over the batch        */
} msp_tune_point;
int msp_autotune(msp_ctx *ctx, int batch, const msp_batch_desc *desc, const int32_t *A_dev,
                 const int64_t *d_dev, int mode, int order, const msp_params *base, msp_params *best,
                 msp_tune_point *points, int *npoints, void *stream);

/* The root count msp_autotune tuned for instances of shape (m, n) in `mode` on
 * this context's device, in *target_roots; 0 if that shape was not tuned.
 * Errors: MSP_E_ARG. */
int msp_tune_lookup(msp_ctx *ctx, int mode, int m, int n, int *target_roots);

/* ---- root traces and the root-scoring model (a project addition; none of
 * this is in the paper) ------------------------------------------------- */

/* Exhaustive msp_enumerate (MSP_ALL, plain order) that also returns, for
 * every subtree root at the split level, MSP_NFEAT features (feat_dev, FP32
 * row-major, cap_roots x MSP_NFEAT) and a label (label_dev, uint8: 1 iff a
 * solution lies in that root's subtree).  Features of root r at level L with
 * prefix u_{k-1..L}, partial norm l, projected vector w (R = n+1):
 *   0 l/R   1 l/||w||_1   2 min(||w||_inf,4)/4   3 mean zig-zag rank of u_j
 *   4 fraction of levels with rank > 0   5 min(max rank,8)/8
 *   6 fraction of u_j != 0   7 mean |u_j|   8 min(max|u_j|,4)/4
 *   9 x_L^2 beta_L / R   10 min(|x_L|,2)/2   11 (L/k) ln(max((R-l)/R,1e-6))/8
 *   12 r / roots   13 fraction of |w_j| > 17/16   14 L/k   15 m/16
 * (rank of u_j = its position in level j's zig-zag sequence; u_j itself while
 * all higher u are 0).  *nroots = root count, *n_found = solutions.
 * Errors: those of msp_enumerate; MSP_E_CAPACITY if roots > cap_roots (only
 * *nroots is set) or more than 65536 solutions (labels incomplete). */
int msp_root_trace(msp_ctx *ctx, int m, int n, const int32_t *A_dev, const int64_t *d_dev,
                   const int64_t *basis_dev, int k, const msp_params *p, float *feat_dev,
                   uint8_t *label_dev, int64_t cap_roots, int64_t *nroots, int64_t *n_found,
                   msp_stats *stats, void *stream);

/* Model weights (host arrays of MSP_MODEL_NPARAM floats, FP32 master copy).
 * msp_model_init: He-normal hidden weights, N(0,1/64) output weights, zero
 * biases, from `seed`.  msp_model_set rejects non-finite values (MSP_E_ARG).
 * msp_model_get: MSP_E_ARG if no model was set. */
int msp_model_init(msp_ctx *ctx, uint64_t seed);
int msp_model_set(msp_ctx *ctx, const float *w);
int msp_model_get(msp_ctx *ctx, float *w);

/* logit_dev[i] = model score of feature row i (count rows, device arrays). */
int msp_model_score(msp_ctx *ctx, const float *feat_dev, int64_t count, float *logit_dev, void *stream);

/* Gradient (grad_dev, MSP_MODEL_NPARAM floats, device) and value (*loss,
 * host) of the weighted logistic loss over all `count` rows:
 *   loss = (1/count) sum_i c_i (softplus(z_i) - y_i z_i),
 *   c_i = pos_weight if label_i = 1 else 1. */
int msp_model_grad(msp_ctx *ctx, const float *feat_dev, const uint8_t *label_dev, int64_t count,
                   float pos_weight, float *grad_dev, float *loss, void *stream);

typedef struct {
    int epochs;        /* passes over the data                               [20] */
    int batch;         /* rows per optimizer step, a multiple of 64        [8192] */
    float lr;          /* Adam step size                                   [1e-3] */
    float pos_weight;  /* weight of label-1 rows; <= 0: negatives/positives  [0] */
    uint64_t seed;     /* epoch shuffles                                      [1] */
    int use_graph;     /* 1: replay each epoch's launches as one HIP graph    [1] */
} msp_train_params;
int msp_train_params_default(msp_train_params *tp);

/* Train the model by Adam (beta 0.9/0.999, eps 1e-8; fresh optimizer state
 * each call) on the mean weighted logistic loss of shuffled mini-batches.
 * loss_per_epoch (host, epochs floats, may be NULL) receives each epoch's
 * mean batch loss. */
int msp_model_train(msp_ctx *ctx, const float *feat_dev, const uint8_t *label_dev, int64_t count,
                    const msp_train_params *tp, float *loss_per_epoch, void *stream);

/* Human-readable name of a status code (static storage). */
const char *msp_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* MSP_H */
