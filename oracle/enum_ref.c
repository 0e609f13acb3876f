/*
 * CPU oracle, part 2: the recursive lattice-point enumeration of Algorithm 1
 * (paper, Section 2), written as plainly as possible.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg load this library; the GPU product path never
 * does.  It shares no code with the GPU library.
 *
 * Built with -O2 -ffp-contract=off: every product and sum is rounded on its
 * own, exactly as written.  Each recursion level receives the parent's
 * projected vector w' by value (its own copy), as in Algorithm 1.
 *
 * The level-t step (Section 2, "First/Second pruning condition", Alg. 1):
 *   y_t  = sum_{i>t} u_i mu_{i,t}          centre of level t is c = -y_t,
 *                                          one running sum, i = t+1 .. k-1
 *   x    = u_t + y_t
 *   l    = x^2 beta_t + l'                 ||w^(t)||^2 by the recurrence
 *   prune (return) when l > R (1 + eps)    R = (n+1) r_max^2
 *   w    = x b_hat_t + w'
 *   t > 0: Hoelder test  l > r_max ||w||_1 (1 + eps)   (Thm 2, y = e_t)
 *          first failure: one more zig-zag step, then one direction only;
 *          second failure: return
 *   t = 0: exact leaf check (Thm 1) in integers, then A x = d.
 *
 * Readings of points the paper leaves open (all listed in the design notes):
 *   - values of u_t follow the zig-zag around c: u1 = rint(c) (ties to
 *     even), first step s = +1 if u1 - c <= 0 else -1, then u1+s, u1-s,
 *     u1+2s, ...; after a child returns (or a leaf is checked) u_t advances
 *     to the next value of that sequence, or by dir in one-direction mode;
 *   - the sign symmetry v <-> -v is broken: while every u_i above t is 0,
 *     only u_t = 0, 1, 2, ... is tried, and the first Hoelder failure there
 *     ends the level (its mirror image fails as well);
 *   - the centre y_t is one running sum over i = t+1, t+2, ..., k-1 starting
 *     at 0.0, in the index order Algorithm 1 writes it, every product and
 *     sum rounded on its own;
 *   - eps = 1e-9 relative slack on both tests (solutions lie exactly on the
 *     l2 bound);
 *   - the r_max coordinate is the last one (index n): a solution has
 *     |v_n| = r_max and |v_j| <= r_max (Thm 1), and x_j = (v_j + r_max) / (2 c_j)
 *     after normalising the sign so that v_n = +r_max (binary: r_max = c_j = 1).
 *
 * Counters: eval = a candidate whose l was computed; node = a candidate
 * that passed the l2 test; expansion = a node that passed the Hoelder test
 * and was descended into (t > 0); leaf = a node at t = 0.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#define ORC_MAXK 160
#define ORC_MAXDIM 160

typedef struct {
    int k, dim, m, n;
    const double *bhat;     /* k x dim, row i = b_hat_i                     */
    const double *mu;       /* k x k, mu[i*k + j] = mu_{i,j} for j < i       */
    const double *beta;     /* k, beta_i = ||b_hat_i||^2                     */
    const int64_t *basis;   /* k x dim integer kernel basis                  */
    const int32_t *A;       /* m x n                                         */
    const int64_t *d;       /* m                                             */
    double R, eps;
    int rmax;
    int hoelder;            /* 1: apply the Hoelder test                     */
    int onedir;             /* 1: apply the one-direction cut                */
    int mode;               /* 0: all solutions, 1: stop at the first        */
    int split;              /* split depth s: roots are expanded nodes at level k-s */
    int nthreads;
    int64_t cap;            /* rows available in sol                          */
    double time_cap_s;      /* <= 0: none                                    */
    /* outputs */
    uint8_t *sol;           /* cap x n                                       */
    int64_t *n_found;       /* number of distinct solutions found            */
    int64_t *counters;      /* [0] evals [1] nodes [2] expansions [3] leaves  */
    int64_t *level_counts;  /* optional, k x 3: evals, nodes, expansions      */
    int64_t *n_roots;       /* number of subtree roots generated             */
    int *timed_out;
    const int64_t *cvec;    /* n, c_j = r_max / r_j for bounded variables;
                             * NULL: binary (r_max = c_j = 1)                 */
    int disc_budget;        /* limited discrepancy search: the discrepancies
                             * of a path sum to at most this; < 0: no limit   */
    int disc_count;         /* 0: a value's discrepancy is its rank in the
                             * level's value order; 1: it is 1 for every value
                             * but the level's first (a count of departures) */
} orc_args;

/* Subtree roots, stored flat: root r has prefix u[r*k + i] (i >= level),
 * projected vector w[r*dim + j], partial norm l[r], and the top-zero flag. */
typedef struct {
    int *u;
    double *w;
    double *l;
    int *topzero;
    int *dsc;               /* discrepancies on the root's prefix            */
    int64_t n, cap;
} orc_roots;

typedef struct {
    const orc_args *a;
    int u[ORC_MAXK];
    int64_t cnt[4];
    int64_t *lvl;           /* k x 3 or NULL */
    /* root collection (only while generating roots) */
    int collect_level;      /* -1: none */
    orc_roots roots;
    int oom;
} orc_walker;

typedef struct {
    const orc_args *a;
    const orc_roots *roots;
    int64_t next;           /* atomic cursor */
    volatile int stop;
    pthread_mutex_t lock;
    struct timespec t0;
    int64_t cnt[4];
    int64_t *lvl;
} orc_shared;

static orc_shared *g_sh;    /* set for the duration of one call */

/* Exact leaf test (Thm 1) plus the independent check A x = d. */
static void leaf(orc_walker *W) {
    const orc_args *a = W->a;
    int k = a->k, dim = a->dim, n = a->n, m = a->m;
    int64_t v[ORC_MAXDIM];
    for (int j = 0; j < dim; ++j) {
        int64_t s = 0;
        for (int i = 0; i < k; ++i) s += (int64_t)W->u[i] * a->basis[(int64_t)i * dim + j];
        v[j] = s;
    }
    if (v[n] != a->rmax && v[n] != -a->rmax) return;
    int64_t sg = v[n] > 0 ? 1 : -1;
    uint8_t x[ORC_MAXDIM];
    for (int j = 0; j < n; ++j) {
        int64_t vj = sg * v[j];
        if (vj > a->rmax || vj < -a->rmax) return;
        /* v_j = 2 c_j x_j - r_max (eq. (2) with v_n = r_max) */
        const int64_t cj = a->cvec ? a->cvec[j] : 1;
        const int64_t tj = vj + a->rmax;
        if (tj % (2 * cj) != 0) return;
        x[j] = (uint8_t)(tj / (2 * cj));
    }
    for (int i = 0; i < m; ++i) {
        int64_t s = 0;
        for (int j = 0; j < n; ++j) s += (int64_t)a->A[(int64_t)i * n + j] * x[j];
        if (s != a->d[i]) return;
    }
    pthread_mutex_lock(&g_sh->lock);
    int64_t idx = *a->n_found;
    if (idx < a->cap) memcpy(a->sol + idx * n, x, (size_t)n);
    *a->n_found = idx + 1;
    if (a->mode == 1) g_sh->stop = 1;
    pthread_mutex_unlock(&g_sh->lock);
}

static void roots_free(orc_roots *R) {
    free(R->u); free(R->w); free(R->l); free(R->topzero); free(R->dsc);
    memset(R, 0, sizeof(*R));
}

static int roots_grow(orc_roots *R, int k, int dim) {
    int64_t nc = R->cap ? 2 * R->cap : 1024;
    int *nu = (int *)realloc(R->u, (size_t)nc * (size_t)k * sizeof(int));
    if (nu) R->u = nu;
    double *nw = (double *)realloc(R->w, (size_t)nc * (size_t)dim * sizeof(double));
    if (nw) R->w = nw;
    double *nl = (double *)realloc(R->l, (size_t)nc * sizeof(double));
    if (nl) R->l = nl;
    int *nz = (int *)realloc(R->topzero, (size_t)nc * sizeof(int));
    if (nz) R->topzero = nz;
    int *nd = (int *)realloc(R->dsc, (size_t)nc * sizeof(int));
    if (nd) R->dsc = nd;
    if (!nu || !nw || !nl || !nz || !nd) return -1;
    R->cap = nc;
    return 0;
}

static void push_root(orc_walker *W, const double *w, double l, int topzero, int dsc) {
    const int k = W->a->k, dim = W->a->dim;
    orc_roots *R = &W->roots;
    if (R->n == R->cap && roots_grow(R, k, dim) != 0) { W->oom = 1; g_sh->stop = 1; return; }
    int64_t r = R->n++;
    memcpy(R->u + r * k, W->u, sizeof(int) * (size_t)k);
    memcpy(R->w + r * dim, w, sizeof(double) * (size_t)dim);
    R->l[r] = l;
    R->topzero[r] = topzero;
    R->dsc[r] = dsc;
}

static void check_time(orc_walker *W) {
    const orc_args *a = W->a;
    if (a->time_cap_s <= 0) return;
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    double el = (double)(ts.tv_sec - g_sh->t0.tv_sec) + 1e-9 * (double)(ts.tv_nsec - g_sh->t0.tv_nsec);
    if (el > a->time_cap_s) { g_sh->stop = 1; *a->timed_out = 1; }
}

/* Next value of the zig-zag sequence u1, u1+s, u1-s, u1+2s, ... given the
 * current offset o = u - u1. */
static int zig_next(int o, int s) {
    if (o == 0) return s;
    if ((o > 0) == (s > 0)) return -o;
    return -o + s;
}

/* Centre sum y_t = sum_{i=t+1}^{k-1} u_i mu_{i,t} (Algorithm 1), one running
 * sum in that index order. */
static double centre(const orc_args *a, const int *u, int t) {
    const int k = a->k;
    double y = 0.0;
    for (int i = t + 1; i < k; ++i) y = y + (double)u[i] * a->mu[(int64_t)i * k + t];
    return y;
}

/* Rank of u in its level's value order (Section 3, limited discrepancy
 * search: a discrepancy is a departure from the value order, counted here as
 * how far down the order the value lies).  On a top-zero level the order is
 * 0, 1, 2, ... and the rank is u; otherwise the order is u1, u1+s, u1-s,
 * u1+2s, ... and u1 + o has rank 2|o|-1 when o has the sign of s, else 2|o|.
 * Values reached in one direction after a Hoelder failure keep their rank in
 * that order, so ranks never decrease along a level. */
static int zig_rank(int u, int u1, int s, int topzero) {
    if (topzero) return u;
    const int o = u - u1;
    if (o == 0) return 0;
    const int ao = o < 0 ? -o : o;
    return ((o > 0) == (s > 0)) ? 2 * ao - 1 : 2 * ao;
}

/* dsc: discrepancies on the path above level t.  A value costs its rank
 * (reading "rank") or 1 for any value but the first of the level (reading
 * "count", the number of departures from the heuristic's choice).  With a
 * budget, a level stops at the first value whose cost would take the path
 * beyond it; under either reading every later value of the level costs at
 * least as much. */
static void enum_level(orc_walker *W, int t, const double *wpar, double lpar, int topzero, int dsc) {
    const orc_args *a = W->a;
    const int dim = a->dim;
    double w[ORC_MAXDIM];
    const double y = centre(a, W->u, t);
    const double c = -y;
    const double bound = a->R * (1.0 + a->eps);
    int u1, s, off = 0, onedir, dir;
    if (topzero) {
        u1 = 0; s = 1; onedir = 1; dir = 1;          /* 0, 1, 2, ... */
    } else {
        u1 = (int)rint(c);
        s = ((double)u1 - c <= 0.0) ? 1 : -1;
        onedir = 0; dir = 0;
    }
    int u = u1;
    for (;;) {
        if (g_sh->stop) { W->u[t] = 0; return; }
        const int r0 = zig_rank(u, u1, s, topzero);
        const int rank = a->disc_count ? (r0 > 0) : r0;
        if (a->disc_budget >= 0 && dsc + rank > a->disc_budget) break;
        const double x = (double)u + y;
        const double l = x * x * a->beta[t] + lpar;
        W->cnt[0]++;
        if (W->lvl) W->lvl[t * 3 + 0]++;
        if (l > bound) break;
        W->cnt[1]++;
        if (W->lvl) W->lvl[t * 3 + 1]++;
        if ((W->cnt[1] & 0xFFFFF) == 0) check_time(W);
        const double *bh = a->bhat + (int64_t)t * dim;
        for (int j = 0; j < dim; ++j) w[j] = x * bh[j] + wpar[j];
        W->u[t] = u;
        if (t > 0) {
            int fail = 0;
            if (a->hoelder) {
                double h = 0.0;
                for (int j = 0; j < dim; ++j) h += fabs(w[j]);
                fail = l > (double)a->rmax * h * (1.0 + a->eps);
            }
            if (fail) {
                if (!a->onedir) goto advance;       /* variant: skip the value only */
                if (onedir) break;                  /* second failure: step back     */
                off = zig_next(off, s);             /* one more regular next()       */
                u = u1 + off;
                onedir = 1;
                dir = ((double)u - c > 0.0) ? 1 : -1;
                continue;
            }
            W->cnt[2]++;
            if (W->lvl) W->lvl[t * 3 + 2]++;
            if (W->collect_level == t) {
                push_root(W, w, l, topzero && u == 0, dsc + rank);
            } else {
                enum_level(W, t - 1, w, l, topzero && u == 0, dsc + rank);
            }
        } else {
            W->cnt[3]++;
            leaf(W);
        }
    advance:
        if (onedir) {
            u += dir;
        } else {
            off = zig_next(off, s);
            u = u1 + off;
        }
    }
    W->u[t] = 0;
}

static void *worker(void *arg) {
    orc_walker *W = (orc_walker *)arg;
    const orc_args *a = W->a;
    const int L = a->k - a->split;          /* roots live at level L */
    const orc_roots *R = g_sh->roots;
    for (;;) {
        if (g_sh->stop) break;
        int64_t i = __atomic_fetch_add(&g_sh->next, 1, __ATOMIC_RELAXED);
        if (i >= R->n) break;
        memset(W->u, 0, sizeof(W->u));
        for (int j = L; j < a->k; ++j) W->u[j] = R->u[i * a->k + j];
        enum_level(W, L - 1, R->w + i * a->dim, R->l[i], R->topzero[i], R->dsc[i]);
        check_time(W);
    }
    pthread_mutex_lock(&g_sh->lock);
    for (int c = 0; c < 4; ++c) g_sh->cnt[c] += W->cnt[c];
    if (g_sh->lvl && W->lvl)
        for (int c = 0; c < a->k * 3; ++c) g_sh->lvl[c] += W->lvl[c];
    pthread_mutex_unlock(&g_sh->lock);
    return NULL;
}

/* Returns 0 on success, -1 on bad arguments, -2 out of memory. */
int orc_enumerate(orc_args *a) {
    if (a->k < 1 || a->k > ORC_MAXK - 1 || a->dim > ORC_MAXDIM || a->n + 1 != a->dim) return -1;
    if (a->split < 0 || a->split > a->k - 1) return -1;
    if (a->nthreads < 1) a->nthreads = 1;
    orc_shared sh;
    memset(&sh, 0, sizeof(sh));
    sh.a = a;
    pthread_mutex_init(&sh.lock, NULL);
    clock_gettime(CLOCK_MONOTONIC, &sh.t0);
    g_sh = &sh;
    *a->n_found = 0;
    *a->timed_out = 0;
    if (a->level_counts) memset(a->level_counts, 0, sizeof(int64_t) * (size_t)a->k * 3);
    sh.lvl = a->level_counts;

    /* Root generation: the same recursion over levels k-1 .. k-s, recording
     * every expanded node at level k-s (depth-first order). */
    orc_walker gen;
    memset(&gen, 0, sizeof(gen));
    gen.a = a;
    gen.lvl = a->level_counts ? (int64_t *)calloc((size_t)a->k * 3, sizeof(int64_t)) : NULL;
    double w0[ORC_MAXDIM];
    memset(w0, 0, sizeof(w0));
    if (a->split == 0) {
        /* one root: the empty prefix above level k-1 (the whole tree) */
        gen.collect_level = -1;
        if (roots_grow(&gen.roots, a->k, a->dim) != 0) return -2;
        memset(gen.roots.u, 0, sizeof(int) * (size_t)a->k);
        memset(gen.roots.w, 0, sizeof(double) * (size_t)a->dim);
        gen.roots.l[0] = 0.0;
        gen.roots.topzero[0] = 1;
        gen.roots.dsc[0] = 0;
        gen.roots.n = 1;
    } else {
        gen.collect_level = a->k - a->split;
        enum_level(&gen, a->k - 1, w0, 0.0, 1, 0);
        if (gen.oom) { roots_free(&gen.roots); free(gen.lvl); return -2; }
    }
    for (int c = 0; c < 4; ++c) sh.cnt[c] += gen.cnt[c];
    if (sh.lvl && gen.lvl)
        for (int c = 0; c < a->k * 3; ++c) sh.lvl[c] += gen.lvl[c];
    free(gen.lvl);
    *a->n_roots = gen.roots.n;
    sh.roots = &gen.roots;

    /* Subtrees, one thread per worker, roots handed out in order. */
    int nt = a->nthreads;
    pthread_t *th = (pthread_t *)calloc((size_t)nt, sizeof(pthread_t));
    orc_walker *ws = (orc_walker *)calloc((size_t)nt, sizeof(orc_walker));
    if (!th || !ws) { free(th); free(ws); roots_free(&gen.roots); return -2; }
    for (int i = 0; i < nt; ++i) {
        ws[i].a = a;
        ws[i].collect_level = -1;
        ws[i].lvl = a->level_counts ? (int64_t *)calloc((size_t)a->k * 3, sizeof(int64_t)) : NULL;
        pthread_create(&th[i], NULL, worker, &ws[i]);
    }
    for (int i = 0; i < nt; ++i) pthread_join(th[i], NULL);
    for (int i = 0; i < nt; ++i) free(ws[i].lvl);
    for (int c = 0; c < 4; ++c) a->counters[c] = sh.cnt[c];
    free(th);
    free(ws);
    roots_free(&gen.roots);
    pthread_mutex_destroy(&sh.lock);
    g_sh = NULL;
    return 0;
}
