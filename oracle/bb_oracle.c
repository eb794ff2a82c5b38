/*
 * bb_oracle.c -- plain, slow, sequential FP64 CPU oracle for band -> bidiagonal
 * reduction by bulge chasing with successive band reduction.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the GPU
 * path.  Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no FMA
 * contraction, so every sum is evaluated left to right exactly as written;
 * OpenMP only for the wavefront timing variant).
 *
 * What it computes (paper: Sec. III, Algorithm 1 and its description; the
 * dependency discussion in Sec. III-A; the storage paragraph of Sec. IV):
 *   A is n x n upper banded with b super-diagonals.  The bandwidth is reduced
 *   in stages of TW ("inner tilewidth", Alg. 1 outer loop): a stage with
 *   bandwidth b uses tw = min(TW, b-1) and leaves bandwidth c = b - tw; stages
 *   repeat until c = 1 (bidiagonal).  Within a stage, sweep r (Alg. 1 second
 *   loop) first annihilates the tw entries A[r, r+c+1 .. r+b] with a right
 *   (row) Householder reflector, which creates a bulge below the diagonal whose
 *   left-most column is annihilated with a left (column) reflector (Alg. 1
 *   third loop, two HH lines).  That left reflector creates a new row bulge
 *   b rows further down, which the next step of the same sweep chases.  Only
 *   the first row/column of each bulge is chased; the rest is left for later
 *   sweeps (Sec. III, "excess bulges ... deferred").  Fill therefore stays
 *   within tw sub-diagonals and b+tw super-diagonals, which is the band height
 *   b + 2 tw + 1 stated in the storage paragraph of Sec. IV.
 *
 *   Step geometry (0-based; the paper omits index details in Alg. 2):
 *     step 0 : row k = r, pivot p = r + c, m = min(r+b, n-1) - p  (sweep exists iff m >= 1)
 *     step j : row k = r + c + (j-1) b, pivot p = k + b, m = min(tw, n-1-p); stop when m < 1
 *   Each step: right reflector from A[k, p..p+m], applied to rows k+1..p+m;
 *   then left reflector from A[p..p+m, p], applied to columns p+1..min(p+m+b, n-1).
 *
 *   Householder convention (the paper defers it to its tile-QR reference; we
 *   take the LAPACK xLARFG definition): x = (alpha, x2); if ||x2|| == 0 then
 *   H = I (tau = 0, beta = alpha); else beta = -sign(alpha) ||x|| with
 *   sign(0) = +1, tau = (beta - alpha) / beta, v = x / (alpha - beta), v0 = 1,
 *   and H = I - tau v v^T maps x to beta e1.  The annihilated entries are
 *   written as exact zeros and beta is stored in place.
 */
#define _POSIX_C_SOURCE 200809L
#include <math.h>
#include <omp.h>
#include <sched.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define BBO_MAXTW 4096

typedef struct {
    int64_t n, ldw, uo;   /* element (i,q) lives at w[(i - q + uo) + q * ldw] */
    double *w;
} bbo_band;

static inline double *at(const bbo_band *B, int64_t i, int64_t q) {
    return &B->w[(i - q + B->uo) + q * B->ldw];
}

/* Euclidean norm, reference LAPACK (>= 3.10) xNRM2: Blue's algorithm with the
 * safe-scaling constants of Anderson (ACM TOMS Alg. 978).  Mid-range entries
 * are summed as plain squares left to right; tiny and huge entries go to
 * separately scaled accumulators that are combined at the end. */
static double nrm2(const double *x, int64_t len) {
    const double tsml = 0x1p-511, tbig = 0x1p486, ssml = 0x1p537, sbig = 0x1p-538;
    int notbig = 1;
    double asml = 0.0, amed = 0.0, abig = 0.0;
    for (int64_t t = 0; t < len; ++t) {
        double ax = fabs(x[t]);
        if (ax > tbig) {
            double y = ax * sbig;
            abig = abig + y * y;
            notbig = 0;
        } else if (ax < tsml) {
            if (notbig) { double y = ax * ssml; asml = asml + y * y; }
        } else {
            amed = amed + ax * ax;
        }
    }
    double scl, sumsq;
    if (abig > 0.0) {
        if (amed > 0.0 || amed != amed) abig = abig + (amed * sbig) * sbig;
        scl = 1.0 / sbig;
        sumsq = abig;
    } else if (asml > 0.0) {
        if (amed > 0.0 || amed != amed) {
            amed = sqrt(amed);
            asml = sqrt(asml) / ssml;
            double ymin = asml > amed ? amed : asml, ymax = asml > amed ? asml : amed;
            double q = ymin / ymax;
            scl = 1.0;
            sumsq = ymax * ymax * (1.0 + q * q);
        } else {
            scl = 1.0 / ssml;
            sumsq = asml;
        }
    } else {
        scl = 1.0;
        sumsq = amed;
    }
    return scl * sqrt(sumsq);
}

/* Exported for the pins of the norm itself (tests call it directly). */
double bbo_nrm2(const double *x, int64_t len) { return nrm2(x, len); }

/* sqrt(a^2 + b^2) without avoidable overflow (LAPACK xLAPY2). */
static double hypot2(double a, double b) {
    double xa = fabs(a), ya = fabs(b);
    double w = xa > ya ? xa : ya, z = xa < ya ? xa : ya;
    if (z == 0.0) return w;
    double q = z / w;
    return w * sqrt(1.0 + q * q);
}

/* Householder generation (LAPACK xLARFG): x[0..m] in, v[0..m], *tau, *beta out.
 * When |beta| falls below safmin = DBL_MIN / DBL_EPSILON, x is rescaled by
 * 1/safmin (at most 20 times) before tau and v are formed, so that 1/(alpha -
 * beta) cannot overflow; beta is scaled back at the end. */
static void house(const double *x_in, int64_t m, double *v, double *tau, double *beta) {
    double x[BBO_MAXTW + 1];
    for (int64_t t = 0; t <= m; ++t) x[t] = x_in[t];
    double alpha = x[0];
    double xn = nrm2(x + 1, m);
    v[0] = 1.0;
    if (xn == 0.0) {
        for (int64_t t = 1; t <= m; ++t) v[t] = 0.0;
        *tau = 0.0;
        *beta = alpha;
        return;
    }
    double h = hypot2(alpha, xn);
    double bt = (alpha >= 0.0) ? -h : h;
    const double safmin = 2.2250738585072014e-308 / 2.220446049250313e-16;
    const double rsafmn = 1.0 / safmin;
    int knt = 0;
    if (fabs(bt) < safmin) {
        do {
            ++knt;
            for (int64_t t = 1; t <= m; ++t) x[t] = x[t] * rsafmn;
            bt = bt * rsafmn;
            alpha = alpha * rsafmn;
        } while (fabs(bt) < safmin && knt < 20);
        xn = nrm2(x + 1, m);
        h = hypot2(alpha, xn);
        bt = (alpha >= 0.0) ? -h : h;
    }
    double scal = 1.0 / (alpha - bt);
    for (int64_t t = 1; t <= m; ++t) v[t] = x[t] * scal;
    *tau = (bt - alpha) / bt;
    for (int k = 0; k < knt; ++k) bt = bt * safmin;
    *beta = bt;
}

/* dot of a strided sequence with v, in forward or reversed order */
typedef struct { int rev; } bbo_opts;

/* Right (row) task: reflector from A[k, p..p+m], applied to rows k+1..p+m. */
static void task_right(bbo_band *A, int64_t k, int64_t p, int64_t m, const bbo_opts *o,
                       double *V, int64_t ldv) {
    double x[BBO_MAXTW + 1], v[BBO_MAXTW + 1], tau, beta;
    for (int64_t t = 0; t <= m; ++t) x[t] = *at(A, k, p + t);
    house(x, m, v, &tau, &beta);
    *at(A, k, p) = beta;
    for (int64_t t = 1; t <= m; ++t) *at(A, k, p + t) = 0.0;
    if (tau == 0.0) return;
    for (int64_t i = k + 1; i <= p + m; ++i) {
        double w = 0.0;
        if (!o->rev) for (int64_t t = 0; t <= m; ++t) w = w + *at(A, i, p + t) * v[t];
        else         for (int64_t t = m; t >= 0; --t) w = w + *at(A, i, p + t) * v[t];
        double tw = tau * w;
        for (int64_t t = 0; t <= m; ++t) *at(A, i, p + t) = *at(A, i, p + t) - tw * v[t];
    }
    if (V) {  /* V <- V H on columns p..p+m (all rows) */
        for (int64_t i = 0; i < A->n; ++i) {
            double w = 0.0;
            for (int64_t t = 0; t <= m; ++t) w = w + V[i + (p + t) * ldv] * v[t];
            double tw = tau * w;
            for (int64_t t = 0; t <= m; ++t) V[i + (p + t) * ldv] = V[i + (p + t) * ldv] - tw * v[t];
        }
    }
}

/* Left (column) task: reflector from A[p..p+m, p], applied to columns p+1..L. */
static void task_left(bbo_band *A, int64_t b, int64_t p, int64_t m, const bbo_opts *o,
                      double *U, int64_t ldu) {
    double x[BBO_MAXTW + 1], v[BBO_MAXTW + 1], tau, beta;
    int64_t L = p + m + b;
    if (L > A->n - 1) L = A->n - 1;
    for (int64_t t = 0; t <= m; ++t) x[t] = *at(A, p + t, p);
    house(x, m, v, &tau, &beta);
    *at(A, p, p) = beta;
    for (int64_t t = 1; t <= m; ++t) *at(A, p + t, p) = 0.0;
    if (tau == 0.0) return;
    for (int64_t q = p + 1; q <= L; ++q) {
        double w = 0.0;
        if (!o->rev) for (int64_t t = 0; t <= m; ++t) w = w + v[t] * *at(A, p + t, q);
        else         for (int64_t t = m; t >= 0; --t) w = w + v[t] * *at(A, p + t, q);
        double tw = tau * w;
        for (int64_t t = 0; t <= m; ++t) *at(A, p + t, q) = *at(A, p + t, q) - tw * v[t];
    }
    if (U) {  /* U <- U H on columns p..p+m (all rows) */
        for (int64_t i = 0; i < A->n; ++i) {
            double w = 0.0;
            for (int64_t t = 0; t <= m; ++t) w = w + U[i + (p + t) * ldu] * v[t];
            double tw = tau * w;
            for (int64_t t = 0; t <= m; ++t) U[i + (p + t) * ldu] = U[i + (p + t) * ldu] - tw * v[t];
        }
    }
}

/* Step geometry of sweep r, step j in a stage (b, tw, c).  Returns m (< 1: no step). */
static int64_t step_geom(int64_t n, int64_t b, int64_t tw, int64_t c, int64_t r, int64_t j,
                         int64_t *k, int64_t *p) {
    if (j == 0) {
        *k = r;
        *p = r + c;
        int64_t last = r + b < n - 1 ? r + b : n - 1;
        return last - *p;
    }
    *k = r + c + (j - 1) * b;
    *p = *k + b;
    int64_t m = n - 1 - *p;
    return m < tw ? m : tw;
}

static int setup(int64_t n, int64_t *b, int64_t TW, const double *band, int64_t ldband,
                 bbo_band *A, int64_t *tw0) {
    if (n < 0) return -1;
    if (*b < 0) return -2;
    if (TW < 1 || TW > BBO_MAXTW) return -3;
    if (!band && n > 0) return -4;
    if (ldband < *b + 1) return -5;
    int64_t bb = *b;
    if (n > 0 && bb > n - 1) bb = n - 1;
    int64_t tw = bb > 1 ? (TW < bb - 1 ? TW : bb - 1) : 0;
    A->n = n;
    A->uo = bb + tw > 1 ? bb + tw : 1;  /* room for the super-diagonal even when b = 0 */
    A->ldw = A->uo + tw + 1;
    A->w = (double *)calloc((size_t)(A->ldw * (n > 0 ? n : 1)), sizeof(double));
    if (!A->w) return 1;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = (j - bb > 0 ? j - bb : 0); i <= j; ++i)
            *at(A, i, j) = band[(*b + i - j) + j * ldband];
    *b = bb;
    *tw0 = tw;
    return 0;
}

static void extract(const bbo_band *A, double *d, double *e) {
    for (int64_t i = 0; i < A->n; ++i) d[i] = *at(A, i, i);
    for (int64_t i = 0; i + 1 < A->n; ++i) e[i] = *at(A, i, i + 1);
}

/*
 * Sequential reduction: stage by stage, sweep r completely before sweep r+1.
 * band: LAPACK upper band, A(i,j) = band[(b + i - j) + j*ldband], ldband >= b+1.
 * d (n), e (n-1): outputs.  U, V: optional n x n column-major (ld n) arrays that
 * receive the accumulated orthogonal factors, so that U^T A V = bidiag(d, e).
 * rev != 0 evaluates every dot product in reversed order (a sensitivity probe).
 * Returns 0, or -i for an invalid argument i, or 1 on allocation failure.
 */
int bbo_reduce(int64_t n, int64_t b, int64_t TW, const double *band, int64_t ldband,
               double *d, double *e, double *U, double *V, int rev) {
    bbo_band A;
    int64_t tw0;
    int rc = setup(n, &b, TW, band, ldband, &A, &tw0);
    if (rc) return rc;
    if (U) { memset(U, 0, sizeof(double) * n * n); for (int64_t i = 0; i < n; ++i) U[i + i * n] = 1.0; }
    if (V) { memset(V, 0, sizeof(double) * n * n); for (int64_t i = 0; i < n; ++i) V[i + i * n] = 1.0; }
    bbo_opts o = {rev};
    int64_t bs = b;
    while (bs > 1) {
        int64_t tw = TW < bs - 1 ? TW : bs - 1, c = bs - tw;
        for (int64_t r = 0; r + c + 1 <= n - 1; ++r) {
            for (int64_t j = 0;; ++j) {
                int64_t k, p, m = step_geom(n, bs, tw, c, r, j, &k, &p);
                if (m < 1) break;
                task_right(&A, k, p, m, &o, V, n);
                task_left(&A, bs, p, m, &o, U, n);
            }
        }
        bs = c;
    }
    extract(&A, d, e);
    free(A.w);
    return 0;
}

/*
 * Host simulation of a pipelined execution (a race detector without a GPU).
 * Half-step h = 2j is the right task of step j, h = 2j+1 its left task.  Half-
 * step h of sweep r may run once sweep r-1 has completed half-steps 0..h+H-1,
 * or is DONE; a sweep becomes DONE when all its half-steps ran and sweep r-1 is
 * DONE.  H is lag[0] when c == 1, lag[1] when c == 2, lag[2] when c >= 3.  The
 * ready tasks run in an order drawn from a xorshift64 stream seeded by `seed`.
 * If the rule is safe, every such order gives results bitwise equal to
 * bbo_reduce(), because tasks that may run concurrently touch disjoint data.
 * Returns as bbo_reduce, or 2 if the rule deadlocks.
 */
int bbo_reduce_pipelined(int64_t n, int64_t b, int64_t TW, const double *band, int64_t ldband,
                         double *d, double *e, const int *lag, uint64_t seed) {
    bbo_band A;
    int64_t tw0;
    int rc = setup(n, &b, TW, band, ldband, &A, &tw0);
    if (rc) return rc;
    bbo_opts o = {0};
    uint64_t s = seed ? seed : 0x9E3779B97F4A7C15ull;
    int64_t *len = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t *prog = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t *ready = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    const int64_t DONE = INT64_MAX;
    int64_t bs = b;
    while (bs > 1 && rc == 0) {
        int64_t tw = TW < bs - 1 ? TW : bs - 1, c = bs - tw;
        int64_t H = c == 1 ? lag[0] : (c == 2 ? lag[1] : lag[2]);
        int64_t ns = 0;
        for (int64_t r = 0; r + c + 1 <= n - 1; ++r, ++ns) {
            int64_t j = 0, k, p;
            while (step_geom(n, bs, tw, c, r, j, &k, &p) >= 1) ++j;
            len[r] = 2 * j;
            prog[r] = 0;
        }
        int64_t first = 0;  /* lowest sweep not DONE; all below it are DONE */
        while (first < ns) {
            int64_t nr = 0;
            for (int64_t r = first; r < ns; ++r) {
                int dep = (r == 0) || prog[r - 1] == DONE || prog[r - 1] >= prog[r] + H;
                if (prog[r] != DONE && prog[r] < len[r] && dep) ready[nr++] = r;
                if (prog[r] == 0) break;  /* sweeps after an unstarted one cannot start */
            }
            if (nr == 0) { rc = 2; break; }
            s ^= s << 13; s ^= s >> 7; s ^= s << 17;
            int64_t r = ready[s % (uint64_t)nr];
            int64_t h = prog[r], j = h / 2, k, p;
            int64_t m = step_geom(n, bs, tw, c, r, j, &k, &p);
            if (h % 2 == 0) task_right(&A, k, p, m, &o, NULL, 0);
            else task_left(&A, bs, p, m, &o, NULL, 0);
            prog[r] = h + 1;
            /* DONE is transitive: a finished sweep becomes DONE once its predecessor is */
            for (int64_t q = first; q < ns; ++q) {
                if (prog[q] != DONE && prog[q] >= len[q] && (q == 0 || prog[q - 1] == DONE)) prog[q] = DONE;
                if (prog[q] != DONE) break;
            }
            while (first < ns && prog[first] == DONE) ++first;
        }
        bs = c;
    }
    if (rc == 0) extract(&A, d, e);
    free(len); free(prog); free(ready); free(A.w);
    return rc;
}

/*
 * Wavefront execution on host threads: the multi-core CPU timing baseline.
 * The rule of bbo_reduce_pipelined run for real, with consecutive sweeps
 * bundled into groups of G so that the windows one thread loads are reused by
 * the G sweeps of its group before another core needs them.  Within a stage,
 * threads claim groups in increasing order from a shared counter.  A thread
 * passes over its group's sweeps in order again and again, running the next
 * half-step h of every sweep whose predecessor allows it: sweep r-1 has
 * completed h+H half-steps, or it and every sweep before it has finished.  For
 * the group's first sweep the predecessor is the last sweep of the previous
 * group, whose progress that group's thread publishes (release store after the
 * half-step's writes, acquire load by the reader); a group publishes DONE once
 * all its sweeps have finished and the previous group is DONE.  Stages are
 * separated by the end of the parallel region.  Lower groups never wait on
 * higher ones, so the scheme cannot deadlock, and every order it allows gives
 * results bitwise those of bbo_reduce().  G = 1 is the plain one-sweep-per-
 * thread wavefront.  nthreads <= 0 takes OpenMP's default.  max_stages > 0
 * stops after that many stages (a timing sample; d and e are then the
 * diagonal and super-diagonal of a band that is not yet bidiagonal).  Returns
 * as bbo_reduce; *threads_used (if not NULL) receives the team size.
 */
#define BBO_MAXGROUP 256

static void wait_progress(const int64_t *w, int64_t target) {
    unsigned spins = 0;
    while (__atomic_load_n(w, __ATOMIC_ACQUIRE) < target) {
        if (++spins > 4096) { sched_yield(); spins = 0; }
    }
}

int bbo_reduce_wavefront(int64_t n, int64_t b, int64_t TW, const double *band, int64_t ldband,
                         double *d, double *e, const int *lag, int nthreads, int64_t G, int64_t max_stages,
                         int *threads_used) {
    if (G < 1 || G > BBO_MAXGROUP) return -10;
    bbo_band A;
    int64_t tw0;
    int rc = setup(n, &b, TW, band, ldband, &A, &tw0);
    if (rc) return rc;
    const bbo_opts o = {0};
    const int64_t DONE = INT64_MAX;
    enum { PAD = 16 };   /* one progress word per 128 bytes: spinning readers do not share a line */
    const int64_t ngmax = n / G + 2;
    int64_t *pub = (int64_t *)calloc((size_t)ngmax * PAD, sizeof(int64_t));
    if (!pub) { free(A.w); return 1; }
    int team = 1;
    int64_t bs = b;
    for (int64_t stage = 0; bs > 1 && (max_stages <= 0 || stage < max_stages); ++stage) {
        const int64_t tw = TW < bs - 1 ? TW : bs - 1, c = bs - tw;
        const int64_t H = c == 1 ? lag[0] : (c == 2 ? lag[1] : lag[2]);
        const int64_t ns = n - 1 - c > 0 ? n - 1 - c : 0;   /* sweeps r with r + c + 1 <= n - 1 */
        const int64_t ng = (ns + G - 1) / G;
        for (int64_t g = 0; g < ng; ++g) pub[g * PAD] = 0;
        int64_t next = 0;
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : omp_get_max_threads())
        {
#pragma omp single
            team = omp_get_num_threads();
            int64_t lp[BBO_MAXGROUP];   /* half-steps completed by each sweep of the group */
            for (;;) {
                const int64_t g = __atomic_fetch_add(&next, 1, __ATOMIC_RELAXED);
                if (g >= ng) break;
                const int64_t r0 = g * G, gs = ns - r0 < G ? ns - r0 : G;
                int64_t fin = 0;   /* sweeps r0 .. r0+fin-1 have finished */
                for (int64_t i = 0; i < gs; ++i) lp[i] = 0;
                while (fin < gs) {
                    int moved = 0;
                    for (int64_t i = fin; i < gs; ++i) {
                        const int64_t r = r0 + i, h = lp[i];
                        int64_t k, p, m = step_geom(n, bs, tw, c, r, h / 2, &k, &p);
                        if (m < 1) {   /* finished; the finished prefix only grows in order */
                            if (i == fin) ++fin;
                            continue;
                        }
                        /* may half-step h of sweep r run? */
                        int ok;
                        if (i == 0) {
                            ok = g == 0 || __atomic_load_n(&pub[(g - 1) * PAD], __ATOMIC_ACQUIRE) >= h + H;
                        } else {
                            ok = lp[i - 1] >= h + H;
                            if (!ok && fin >= i)   /* every earlier sweep of the group finished */
                                ok = g == 0 || __atomic_load_n(&pub[(g - 1) * PAD], __ATOMIC_ACQUIRE) == DONE;
                        }
                        if (!ok) continue;
                        if (h % 2 == 0) task_right(&A, k, p, m, &o, NULL, 0);
                        else task_left(&A, bs, p, m, &o, NULL, 0);
                        lp[i] = h + 1;
                        moved = 1;
                        if (i == gs - 1) __atomic_store_n(&pub[g * PAD], h + 1, __ATOMIC_RELEASE);
                    }
                    if (!moved && fin < gs) sched_yield();
                }
                if (g > 0) wait_progress(&pub[(g - 1) * PAD], DONE);
                __atomic_store_n(&pub[g * PAD], DONE, __ATOMIC_RELEASE);
            }
        }
        bs = c;
    }
    extract(&A, d, e);
    if (threads_used) *threads_used = team;
    free(pub);
    free(A.w);
    return 0;
}

/*
 * Symmetric variant: band -> tridiagonal for the symmetric eigenvalue problem
 * (the paper names this sister reduction as the one that bulge chasing also
 * serves; it reduces the non-symmetric band to bidiagonal form).  The same
 * successive band reduction and the same step geometry, with one reflector per
 * step applied from both sides, A <- H A H.
 *
 *   A is n x n symmetric with b sub-diagonals, held as its lower triangle:
 *   LAPACK lower band layout A(i, j) = band[(i - j) + j * ldband], 0 <= i - j <= b.
 *   Stage (b, tw, c = b - tw), sweep r, step j: k, p, m as in the bidiagonal
 *   case (step 0: k = r, p = r + c; step j: k = r + c + (j-1) b, p = k + b;
 *   m = min(tw, n-1-p), for step 0 min(r+b, n-1) - p).  The step:
 *     1. reflector from the column segment A[p..p+m, k]; A[p, k] = beta and
 *        A[p+1..p+m, k] = 0 exactly;
 *     2. left application H A on rows p..p+m of columns k+1 .. p+m, where the
 *        (m+1) x (m+1) diagonal block is taken whole (its upper triangle is the
 *        mirror of the stored lower one);
 *     3. right application (H A) H on columns p..p+m of the block's rows and of
 *        rows p+m+1 .. min(p+m+b, n-1);
 *     4. the lower triangle of the block is stored back (its upper triangle,
 *        equal up to rounding, is dropped).
 *   Every dot product is summed left to right; no fused multiply-add.
 *   Output: d = diagonal, e = sub-diagonal of the tridiagonal T = Q^T A Q
 *   (Q e1 = e1; with Q != NULL the n x n column-major Q is accumulated by
 *   Q <- Q H in the order the reflectors are applied).
 */
typedef struct {
    int64_t n, ldw;   /* element (i, q), q <= i <= q + ldw - 1, at w[(i - q) + q * ldw] */
    double *w;
} bbo_sband;

static inline double *sat(const bbo_sband *S, int64_t i, int64_t q) { return &S->w[(i - q) + q * S->ldw]; }

static void sym_step(bbo_sband *S, int64_t b, int64_t k, int64_t p, int64_t m, double *Q) {
    const int64_t n = S->n;
    double x[BBO_MAXTW + 1], v[BBO_MAXTW + 1], tau, beta;
    for (int64_t t = 0; t <= m; ++t) x[t] = *sat(S, p + t, k);
    house(x, m, v, &tau, &beta);
    *sat(S, p, k) = beta;
    for (int64_t t = 1; t <= m; ++t) *sat(S, p + t, k) = 0.0;
    if (tau == 0.0) return;
    const int64_t w1 = m + 1;
    double *B = (double *)malloc(sizeof(double) * (size_t)(w1 * w1));  /* B[s + t*w1] = A(p+s, p+t) */
    for (int64_t t = 0; t < w1; ++t)
        for (int64_t s = 0; s < w1; ++s) B[s + t * w1] = s >= t ? *sat(S, p + s, p + t) : *sat(S, p + t, p + s);
    /* left: columns k+1 .. p-1 (rows p..p+m, all below the diagonal) */
    for (int64_t q = k + 1; q < p; ++q) {
        double w = 0.0;
        for (int64_t t = 0; t <= m; ++t) w = w + v[t] * *sat(S, p + t, q);
        double tw = tau * w;
        for (int64_t t = 0; t <= m; ++t) *sat(S, p + t, q) = *sat(S, p + t, q) - tw * v[t];
    }
    /* left: the block's columns */
    for (int64_t q = 0; q < w1; ++q) {
        double w = 0.0;
        for (int64_t t = 0; t < w1; ++t) w = w + v[t] * B[t + q * w1];
        double tw = tau * w;
        for (int64_t t = 0; t < w1; ++t) B[t + q * w1] = B[t + q * w1] - tw * v[t];
    }
    /* right: the block's rows */
    for (int64_t s = 0; s < w1; ++s) {
        double w = 0.0;
        for (int64_t t = 0; t < w1; ++t) w = w + B[s + t * w1] * v[t];
        double tw = tau * w;
        for (int64_t t = 0; t < w1; ++t) B[s + t * w1] = B[s + t * w1] - tw * v[t];
    }
    /* right: rows p+m+1 .. L */
    int64_t L = p + m + b;
    if (L > n - 1) L = n - 1;
    for (int64_t i = p + m + 1; i <= L; ++i) {
        double w = 0.0;
        for (int64_t t = 0; t <= m; ++t) w = w + *sat(S, i, p + t) * v[t];
        double tw = tau * w;
        for (int64_t t = 0; t <= m; ++t) *sat(S, i, p + t) = *sat(S, i, p + t) - tw * v[t];
    }
    for (int64_t t = 0; t < w1; ++t)
        for (int64_t s = t; s < w1; ++s) *sat(S, p + s, p + t) = B[s + t * w1];
    free(B);
    if (Q) {  /* Q <- Q H on columns p..p+m (all rows) */
        for (int64_t i = 0; i < n; ++i) {
            double w = 0.0;
            for (int64_t t = 0; t <= m; ++t) w = w + Q[i + (p + t) * n] * v[t];
            double tw = tau * w;
            for (int64_t t = 0; t <= m; ++t) Q[i + (p + t) * n] = Q[i + (p + t) * n] - tw * v[t];
        }
    }
}

/*
 * Symmetric band (lower layout, b sub-diagonals, ldband >= b+1) -> tridiagonal
 * (d: n diagonal entries, e: n-1 sub-diagonal entries), inner tilewidth TW.
 * Q (may be NULL): n x n column-major with Q^T A Q = tridiag(d, e).
 * Returns 0, -i for an invalid argument i, or 1 on allocation failure.
 */
int bbo_sym_reduce(int64_t n, int64_t b, int64_t TW, const double *band, int64_t ldband, double *d, double *e,
                   double *Q) {
    if (n < 0) return -1;
    if (b < 0) return -2;
    if (TW < 1 || TW > BBO_MAXTW) return -3;
    if (!band && n > 0) return -4;
    if (ldband < b + 1) return -5;
    int64_t bb = b;
    if (n > 0 && bb > n - 1) bb = n - 1;
    int64_t tw0 = bb > 1 ? (TW < bb - 1 ? TW : bb - 1) : 0;
    bbo_sband S;
    S.n = n;
    S.ldw = bb + tw0 + 2;  /* rows q .. q + b + tw of column q (fill), plus the sub-diagonal when b = 0 */
    S.w = (double *)calloc((size_t)(S.ldw * (n > 0 ? n : 1)), sizeof(double));
    if (!S.w) return 1;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = j; i <= j + bb && i < n; ++i) *sat(&S, i, j) = band[(i - j) + j * ldband];
    if (Q) { memset(Q, 0, sizeof(double) * n * n); for (int64_t i = 0; i < n; ++i) Q[i + i * n] = 1.0; }
    int64_t bs = bb;
    while (bs > 1) {
        int64_t tw = TW < bs - 1 ? TW : bs - 1, c = bs - tw;
        for (int64_t r = 0; r + c + 1 <= n - 1; ++r) {
            for (int64_t j = 0;; ++j) {
                int64_t k, p, m = step_geom(n, bs, tw, c, r, j, &k, &p);
                if (m < 1) break;
                sym_step(&S, bs, k, p, m, Q);
            }
        }
        bs = c;
    }
    for (int64_t i = 0; i < n; ++i) {
        d[i] = *sat(&S, i, i);
        if (i + 1 < n) e[i] = *sat(&S, i + 1, i);
    }
    free(S.w);
    return 0;
}
