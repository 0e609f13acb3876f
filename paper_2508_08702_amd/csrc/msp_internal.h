// Internal declarations shared by the HIP translation units of libmsp.
// Every kernel is launched from a host wrapper in the file that defines it;
// the wrappers below are what the C ABI layer (api.hip) calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msp {

// Root / frontier record layout (structure of arrays, one entry per record):
//   u   int8  [cap x k]   prefix u_i for levels >= the record's level, 0 below
//   w   f64   [cap x WS]  projected vector w^(level) in natural column order,
//                         zero padded to DIMP columns, then a copy of columns
//                         0..WS-DIMP-1 (so that a lane rotated by r can read
//                         w[r .. r+DIMP) without wrapping)
//   l   f64   [cap]       ||w||^2 by the partial-norm recurrence
//   tz  uint8 [cap]       1 while every u above the record's level is zero
//   dsc uint8 [cap]       discrepancies on the prefix: the sum of the ranks of
//                         its values in their levels' value orders (limited
//                         discrepancy search, paper Section 3), capped at 255
// Records of one level of the frontier.  The projected vectors are stored
// column-major: element j of record r at w[j * wcap + r] (wcap = the buffer's
// record capacity), so a thread per record reads and writes them coalesced.
struct Frontier {
    int8_t *u;
    double *w;
    double *l;
    uint8_t *tz;
    uint8_t *dsc;
    int64_t wcap;
};

inline int dimp_for(int dim) {
    // supported compile-time widths (even, ascending)
    static const int widths[] = {24, 32, 40, 48, 52, 56, 64, 72, 82, 88, 96, 102, 112, 128};
    for (int w : widths)
        if (dim <= w) return w;
    return -1;
}

struct GsArgs {
    int k, dim;
    const int64_t *basis;   // k x dim
    double *bhat;           // k x dim
    double *mu;             // k x k
    double *beta;           // k
    int *err;               // set to 1 on a non-positive norm
};
hipError_t launch_gram_schmidt(const GsArgs &a, hipStream_t st);

struct ExpandArgs {
    int k, dim, dimp, ws, t;       // t: level whose candidates are enumerated
    const double *bhat, *mu, *beta;
    Frontier par;                  // parents: expanded nodes of level t+1
    int64_t np;
    Frontier ch;                   // children (write pass only)
    const int64_t *offs;           // write pass: first child slot per parent
    int64_t *counts;               // count pass: children per parent
    double bound, hfac;            // l2 bound R (1 + eps); Hoelder: l > (rmax h) hfac
    double rmax;                   // r_max (1 for binary variables)
    int budget;                    // discrepancy budget (< 0: none)
    int disc_count;                // 1: a discrepancy costs 1 (count reading), 0: its rank
    int hoelder, onedir;
    unsigned long long *counters;  // [0] evals [1] nodes [2] expansions (write pass)
    int *flags;                    // [1] |u| > 127 seen
};
hipError_t launch_expand_count(const ExpandArgs &a, hipStream_t st);
hipError_t launch_expand_write(const ExpandArgs &a, hipStream_t st);
hipError_t launch_frontier_init(Frontier f, int k, int ws, hipStream_t st);
// exclusive prefix sum of counts[0..n) into offs, total into *total
// Exclusive scan of counts[0..n) into offs and their sum into *total (device).
// temp == nullptr: only sets *temp_bytes, the scratch the scan needs for n.
hipError_t launch_scan(void *temp, size_t *temp_bytes, const int64_t *counts, int64_t *offs, int64_t n,
                       int64_t *total, hipStream_t st);

// Work-item pool of the walker: item i = (level T, prefix u_{T+1..k-1},
// zig-zag continuation at level T).
//   u     int8 [cap x k]  prefix (natural level index; entries <= T are 0)
//   meta  int4 [cap]      {T, u_start, flags (onedir 1, dir>0 2, topzero 4,
//                          fresh 8: start the level from its first value),
//                          discrepancies on the prefix above level T}
//   ready int  [cap]      set (release) once a donated item is fully written
struct Pool {
    int8_t *u;
    int4 *meta;
    int *ready;
    int *root;  // donated items: the root they descend from (index into the root arrays), or -1
    int64_t cap;
};

struct WalkArgs {
    int k, dim, n, m, L;           // L: split level; walkers live on levels < L
    const double *g_bh;            // k x S rotated rows (see walk.hip)
    const double *g_muc;           // mu by columns, column t at g_coff[t]
    const int *g_coff;             // k + 1 column offsets
    int muc_len;                   // doubles in g_muc
    const double *beta;            // k
    const int64_t *basis;          // k x dim, exact leaf reconstruction
    const int32_t *A;
    const int64_t *d;
    Pool pool;
    int64_t nroots;                // items 0..nroots-1 come from root generation
    const double *root_w;          // their projected vectors (frontier layout: element j of root r at
    int64_t root_wcap;             //   root_w[j * root_wcap + r], j < DIMP)
    const double *root_l;          // their partial norms
    int root_level;                // the roots' level: their w includes levels root_level .. k-1
    const int64_t *order;          // optional permutation of those (nullptr = identity)
    unsigned long long *head;      // next ticket
    unsigned long long *tail;      // next free pool slot
    long long *pending;            // items created and not yet finished
    double *stack;                 // per walker k entries x 4 doubles
    uint8_t *x_out;
    uint8_t *leaf_x;               // per walker n bytes: a leaf's x staged while it is checked
    int8_t *sol_u;                 // optional: u_0..u_{k-1} of each written solution (cap x k)
    int64_t cap;
    unsigned long long *n_found;
    unsigned long long *counters;  // [0] evals [1] nodes [2] expansions [3] leaves [4] items done
    int *flags;                    // [0] stop [1] overflow [2] timeout [3] internal error
    unsigned long long *t_first;   // wall clock of the first verified hit (0 = none)
    unsigned long long *t_start;   // wall clock when the kernel started
    unsigned long long deadline;   // time cap in wall-clock ticks from kernel start (0 = none)
    int mode;                      // 0 all, 1 first
    double bound, hfac;            // l2 bound R (1 + eps); Hoelder: l > (rmax h) hfac
    double rmax_d;                 // r_max as a double
    long long rmax;                // r_max: a solution has v_n = +-r_max, |v_j| <= r_max
    const int64_t *cvec;           // c_j = r_max / r_j (nullptr: binary, c_j = 1)
    int budget;                    // discrepancy budget (< 0: none)
    int disc_count;                // 1: a discrepancy costs 1 (count reading), 0: its rank
    int hoelder, onedir;
};
hipError_t launch_walk(const WalkArgs &a, int dimp, int block, int num_cus, hipStream_t st);
// block: threads per workgroup of the walk that follows (it fixes the row layout)
hipError_t launch_walk_prep(int k, int dim, int dimp, int block, const double *bhat, const double *mu,
                            double *g_bh, double *g_muc, int *g_coff, hipStream_t st);
size_t walk_lds_bytes(int dimp, int block, int k, int L, int muc_len);
__host__ __device__ int walk_row_stride(int dimp, int block);  // doubles per LDS row
int walk_muc_len(int k);
int walk_block_for(int dimp, int k, int L);  // 0 when no variant fits
int walk_max_level(int dimp, int k);         // largest split level whose walker fits in LDS

hipError_t launch_pool_init(Frontier f, int64_t nroots, int k, int L, Pool pool, hipStream_t st);
// dst record r = src record idx[r] (idx == nullptr: base + r), r < n
hipError_t launch_gather_frontier(Frontier src, const int64_t *idx, int64_t base, int64_t n, Frontier dst, int k,
                                  int ws, hipStream_t st);
hipError_t launch_frontier_items(Frontier src, const int64_t *idx, int64_t n, int k, int L, int8_t *iu, int4 *imeta,
                                 hipStream_t st);
hipError_t launch_fill_int(int *p, int64_t n, int v, hipStream_t st);

// ---- root orders and the root-scoring MLP (order.hip) ----
constexpr int kNumFeat = 16;      // features per root
constexpr int kHidden = 64;       // width of both hidden layers
constexpr int kNumParams = kHidden * kNumFeat + kHidden + kHidden * kHidden + kHidden + kHidden + 1;
constexpr int kPartialStride = kNumParams + 7;
constexpr int64_t kTraceSolutions = 1 << 16;  // solutions recorded by a root trace  // floats per partial-gradient row (params + loss, padded)

struct FeatArgs {
    int k, dim, m, L, ws;
    Frontier roots;                // records at level L
    int64_t np;
    const double *mu, *beta;       // Gram-Schmidt data (mu k x k row-major)
    double R;                      // l2 bound n + 1
    float *feat;                   // np x kNumFeat
};
hipError_t launch_root_features(const FeatArgs &a, hipStream_t st);
hipError_t launch_root_labels(Frontier roots, int64_t np, int k, int L, const int8_t *sol_u, int64_t nsol,
                              uint8_t *label, hipStream_t st);
hipError_t launch_disc_keys(const float *feat, int64_t np, int levels, float *key, hipStream_t st);
hipError_t launch_mlp_score(const float *wq, const float *feat, int64_t count, float *logit, hipStream_t st);

struct MlpGradArgs {
    const float *wq;               // BF16-rounded weights
    const float *feat;             // count x kNumFeat
    const uint8_t *label;          // count
    const int32_t *perm;           // sample order (nullptr = identity)
    int64_t count, batch;
    const unsigned long long *step;  // optimizer step counter (nullptr: the batch starting at 0)
    int64_t steps_per_epoch;
    float pos_weight;
    float *partial;                // waves x kPartialStride
};
hipError_t launch_mlp_grad(const MlpGradArgs &a, int waves, hipStream_t st);
hipError_t launch_grad_sum(const float *partial, int waves, float *grad, float *loss, hipStream_t st);

struct AdamArgs {
    float *master, *wq, *m, *v;
    const float *partial;
    int waves;
    unsigned long long *step;
    int64_t steps_per_epoch;
    float lr;
    float *loss_acc;               // per epoch
};
hipError_t launch_adam(const AdamArgs &a, hipStream_t st);  // Adam, then step += 1
hipError_t launch_bf16_round(const float *master, float *wq, hipStream_t st);
hipError_t launch_count_pos(const uint8_t *label, int64_t count, unsigned long long *npos, hipStream_t st);
hipError_t sort_scores_desc(void *temp, size_t *temp_bytes, const float *key_in, float *key_out, int64_t *idx_in,
                            int64_t *idx_out, int64_t n, hipStream_t st);
hipError_t sort_idx_asc(void *temp, size_t *temp_bytes, const int64_t *in, int64_t *out, int64_t n, hipStream_t st);
hipError_t shuffle_perm(void *temp, size_t *temp_bytes, uint32_t *keys, uint32_t *keys_out, int32_t *idx,
                        int32_t *perm, int64_t n, unsigned long long seed, int epoch, hipStream_t st);

// BKZ of a kernel basis (bkz.hip), one wave, in place.
struct BkzArgs {
    int k, dim;
    int64_t *B;                    // count k x dim kernel bases (device), reduced in place;
    int64_t bstride;               //   basis i starts at B + i * bstride
    int count;                     // bases, one workgroup each
    int beta, tours;               // block size, tour limit
    double delta;                  // Lovasz parameter of the LLL inside
    long long max_nodes;           // enumeration nodes per block SVP
    long long max_lll_iters;       // LLL iterations over the whole run
    int *out;                      // per basis i: [2i] status (0, -4 overflow, -10 iteration cap),
                                   //   [2i+1] insertions
    long long *nodes;              // per basis: SVP nodes
    int b_in_lds;                  // set by launch_bkz: the basis fits in LDS
};
hipError_t launch_bkz(BkzArgs a, hipStream_t st);

// Shuffled instance copies (restart.hip): out[r] = A[:, perm[r]] (copies x m x n);
// x[s][perm[j]] = xc[s][j] for s < rows.
hipError_t launch_permute_cols(const int32_t *A, int m, int n, const int32_t *perm, int copies, int32_t *out,
                               hipStream_t st);
hipError_t launch_unpermute_rows(const uint8_t *xc, int64_t rows, int n, const int32_t *perm, uint8_t *x,
                                 hipStream_t st);
__host__ __device__ size_t bkz_lds_bytes(int k);

// Per-instance fields are read as base[i * stride] (in 4-byte units), so a
// packed array of descriptor structs serves as the per-instance arrays.
struct LllArgs {
    const int *m, *n;              // per instance
    const int32_t *A;              // packed instances; A of instance i at A + A_off[i] (m x n)
    const int64_t *A_off;
    const int64_t *d;              // d of instance i at d + d_off[i]
    const int64_t *d_off;
    long long N;                   // scale constant of eq. (2)
    double delta;                  // Lovász parameter
    long long max_iters;           // LLL iteration cap
    long long *work;               // basis workspace, instance i at work + work_off[i] ((n+1) x (m+n+1))
    const int64_t *work_off;
    int64_t *out;                  // kernel basis of instance i at out + out_off[i] (k x (n+1))
    const int64_t *out_off;
    const int64_t *cvec;           // bounded variables: c_j = r_max / r_j (nullptr: binary)
    long long rmax;                // r_max (1 when cvec is nullptr)
    int32_t *status;               // 0, -2 (rank), -3 (not isolated), -4 (overflow), -10 (no convergence)
    int32_t *kout;                 // zero-top vectors found
    long long *iters;              // LLL iterations used
    int stride;                    // distance between instances, in 4-byte units
};
hipError_t launch_lll(const LllArgs &a, int ninst, int max_n, hipStream_t st);
// per-instance descriptor of a reduction launch (the kernel reads its fields
// through the strided views of LllArgs)
struct LllDesc {
    int m, n;
    int64_t A_off, d_off, work_off, out_off;
    int32_t status, kout;
    long long iters;
};
// r_max = lcm(r_0..r_{n-1}) and c_j = r_max / r_j; *rmax = -1 when some
// r_j is outside 1..255, -2 when r_max would exceed 2^20
hipError_t launch_bounds_scale(const int32_t *r, int n, int64_t *cvec, long long *rmax, hipStream_t st);
size_t lll_lds_bytes(int n);

// ---- box bounds (box.hip) ----
hipError_t launch_box_setup(int m, int n, const int32_t *A, const int64_t *d, const int32_t *lo, const int32_t *hi,
                            int64_t *d_out, int32_t *r_out, int *status, hipStream_t st);
hipError_t launch_box_shift(int64_t rows, int n, const uint8_t *xs, const int32_t *lo, int32_t *x, hipStream_t st);

}  // namespace msp
