/*
 * bb.h -- C ABI of the MI355X (gfx950) band -> bidiagonal reduction library.
 *
 * The operation (paper: Sec. III, Algorithm 1; problem statement in Sec. I and
 * Sec. III's opening paragraph): given an n x n upper-banded matrix A with b
 * super-diagonals, compute an upper bidiagonal B = U^T A V (U, V orthogonal,
 * U e1 = V e1 = e1) by bulge chasing with two-sided Householder reflectors,
 * reducing the bandwidth in stages of TW (the "inner tilewidth").  Singular
 * values are preserved: sigma(B) = sigma(A).  bb_reduce returns the bidiagonal
 * (d, e); bb_reduce_vectors also forms U and V.
 *
 * Conventions shared by every entry point
 *   - Band layout (input): LAPACK column-major upper band of the storage type,
 *       A(i, j) = band[(b + i - j) + j * ldband],  max(0, j - b) <= i <= j,
 *     ldband >= b + 1.  Entries above row 0 are ignored.  `band` is read only.
 *   - Storage type (bb_dtype_t): BB_F64 -> double, BB_F32 -> float,
 *     BB_F16 -> IEEE binary16.  The band is stored in this type; updates are
 *     computed in FP64 for BB_F64 (sequential sums, no FMA: bitwise the plain
 *     definition) and in FP32 with fused multiply-add dot products for BB_F32
 *     and BB_F16, then rounded to the storage type.  Householder reflectors
 *     (norm, beta, tau) are always generated in FP64.
 *     BB_F16 keeps a power-of-two scale per bandwidth-reduction stage.
 *   - Outputs: d (n doubles) = diagonal, e (n - 1 doubles) = super-diagonal of
 *     B, always FP64.  Signs of d, e are not unique; |d|, |e| are.
 *   - Memory: every array pointer is caller-owned DEVICE memory on the current
 *     HIP device unless stated otherwise.  The library keeps a private working
 *     band (b + 2 TW + 1 rows per column, the height given in Sec. IV) in
 *     stream-ordered device memory drawn from the device's default pool.
 *   - Streams: `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *     asynchronous: results are valid once the stream is synchronised.  Calls
 *     on different streams use separate working memory and are independent.
 *   - Errors: 0 on success; -i if argument i (1-based) is invalid, with no
 *     work enqueued; > 0 for a runtime failure (BB_ERR_*).  Nothing aborts.
 *     A device-side watchdog on every dependency wait turns a stalled pipeline
 *     into BB_ERR_TIMEOUT, reported by bb_stream_status() (one error word per
 *     device).
 *   - Edge cases: n = 0 is a no-op; n = 1 gives d0 = a00; b = 0 gives d =
 *     diagonal, e = 0; b = 1 is copied through; b >= n is treated as n - 1.
 *     NaN / Inf in the input propagate to the output.
 */
#ifndef BB_H
#define BB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { BB_F64 = 0, BB_F32 = 1, BB_F16 = 2 } bb_dtype_t;

enum {
    BB_OK = 0,
    BB_ERR_HIP = 1,          /* a HIP runtime call failed */
    BB_ERR_TIMEOUT = 2,      /* device watchdog: a dependency wait never completed */
    BB_ERR_NOMEM = 3,        /* device or host allocation failed */
    BB_ERR_UNSUPPORTED = 4,  /* parameters outside the compiled kernel variants, or a band
                                column height whose in-window byte offsets would exceed
                                32 bits (working-band columns above about 5.4 million FP64
                                entries; b is far smaller at any size that fits) */
    BB_ERR_NODEVICE = 5,     /* no usable gfx950 device */
    BB_ERR_SCRATCH = 6       /* bb_reduce_noalloc: the call's working memory exceeds the
                                library's static scratch (64 MiB per device) */
};

/*
 * Tuning parameters (Sec. III-C names three knobs: threads per block, inner
 * tilewidth, maximum blocks).  0 in any field means "automatic".
 *   tw                 inner tilewidth TW (entries annihilated per reflector);
 *                      supported values: 1..32 for BB_F64, 1..64 for BB_F32 and
 *                      BB_F16 (a call with a larger value returns
 *                      BB_ERR_UNSUPPORTED).
 *   threads_per_window threads that work on one sweep's window: 64, 128 or 256
 *                      (a stage with tw > 32 uses at least 128).
 *   sweeps_per_group   consecutive sweeps one workgroup advances in lock-step
 *                      (1..16, threads_per_window * sweeps_per_group <= 1024);
 *                      hand-over inside a group costs one workgroup barrier.
 *                      A stage whose kernel variant accepts fewer threads per
 *                      workgroup (256 for tw 17..64, 512 for 9..16) runs fewer
 *                      sweeps per group; results do not depend on it.
 *   groups_per_cu      persistent workgroups launched per compute unit (1..16;
 *                      automatic: 2 for bb_reduce, 4 for bb_reduce_batched);
 *                      with sweeps_per_group it caps the sweeps in flight, the
 *                      paper's "Max blocks".
 *   lag                half-step dependency lag between consecutive sweeps; each
 *                      stage uses max(lag, smallest safe lag of that stage), so
 *                      0 selects the smallest safe value (bb_min_lag) and a
 *                      larger value only delays sweeps (results are unchanged).
 *   xcd_run            consecutive sweep groups placed on one XCD (accelerator
 *                      die with its own L2) before moving to the next (1..4096;
 *                      0 = automatic, 2), so that consecutive sweeps, whose
 *                      windows overlap, share an L2.  Results do not depend on
 *                      it.  bb_reduce only; the batched form claims tasks in one
 *                      global order.
 */
typedef struct {
    int tw;
    int threads_per_window;
    int sweeps_per_group;
    int groups_per_cu;
    int lag;
    int xcd_run;
} bb_params_t;

/*
 * Reduce one upper band to bidiagonal form.
 *   n, b     order and number of super-diagonals (n >= 0, b >= 0).
 *   dtype    storage type of `band` and of the working band.
 *   band     device pointer, LAPACK upper band of `dtype`, ldband >= b + 1.
 *   d, e     device pointers to n and max(n - 1, 0) doubles (outputs).
 *   stream   hipStream_t.
 * Argument numbers for -i: n=1, b=2, dtype=3, band=4, ldband=5, d=6, e=7.
 */
int bb_reduce(int64_t n, int64_t b, bb_dtype_t dtype, const void *band, int64_t ldband,
              double *d, double *e, void *stream);

/*
 * bb_reduce for callers that cannot allocate device memory: code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same arguments,
 * argument numbers, launch parameters and results as bb_reduce (bitwise: the
 * same kernels run in the same configuration); the difference is where the
 * working memory lives.  It is a static device array of 64 MiB that the library
 * holds on every device it runs on until the process ends; this call allocates
 * nothing (no hipMalloc / hipMallocAsync / hipFree, no events) and clears the
 * counters it needs with a kernel at the start of each call.
 *   Limit: the working memory of the call, bb_workspace_bytes(n, b, dtype), must
 *   be at most 64 MiB (it is about 51 MiB for n = 32768, b = 128 in FP64; it
 *   grows with n (b + 2 TW + 1) times the element size); larger shapes return
 *   BB_ERR_SCRATCH with no work enqueued.
 *   Concurrency: every call on one device shares that device's scratch, so calls
 *   that overlap in time on one device (e.g. on two streams) race and give wrong
 *   results; issue them on one stream or otherwise serialise them.  Calls of
 *   bb_reduce and bb_reduce_batched use their own memory and do not conflict.
 */
int bb_reduce_noalloc(int64_t n, int64_t b, bb_dtype_t dtype, const void *band, int64_t ldband,
                      double *d, double *e, void *stream);

/*
 * bb_reduce that also forms the orthogonal factors: U^T A V = bidiag(d, e),
 * U e1 = V e1 = e1.  The paper returns only the bidiagonal and names the
 * singular vectors as the extension (Sec. I, closing paragraph; Sec. VII): the
 * reflectors of the bulge chase are kept (its Algorithm 2 writes each one back
 * in place of the entries it annihilates) and applied afterwards.  Here every
 * reflector (tau, v in FP64, for every storage type) is logged during the
 * reduction and U = H_1 H_2 ... (left reflectors in the order applied), V
 * likewise from the right reflectors, are accumulated from the identity on the
 * device.  d, e are bitwise those of bb_reduce; for BB_F64, U and V equal a plain
 * sequential FP64 accumulation in the reduction's order bitwise (up to the sign
 * of zero).
 *   U, V     device pointers to n x n column-major FP64 matrices with leading
 *            dimensions ldu, ldv >= max(n, 1) (outputs); either may be NULL (not
 *            formed).
 * Other arguments as bb_reduce.  Argument numbers: n=1, b=2, dtype=3, band=4,
 * ldband=5, d=6, e=7, U=8, ldu=9, V=10, ldv=11.  Working memory (stream-ordered,
 * freed by the call) is bb_workspace_bytes plus the reflector log: per stage
 * (b_s, TW_s), 2 (n - c_s - 1)(1 + (n - 2 - c_s) / b_s)(TW + 1) doubles, about
 * 100 MB at n = 2048, b = 64 and 37 GB at n = 32768, b = 128.  The accumulation
 * of stage s's reflectors runs on a second stream that the library owns (one
 * per device, default priority, kept until the process ends) while the
 * reduction continues with the next stage on `stream`; the call orders that
 * stream after the work already queued on `stream` and `stream` after it, so
 * the results, as with every call here, are complete when `stream` reaches the
 * end of the call.
 */
int bb_reduce_vectors(int64_t n, int64_t b, bb_dtype_t dtype, const void *band, int64_t ldband,
                      double *d, double *e, double *U, int64_t ldu, double *V, int64_t ldv,
                      void *stream);

/*
 * Symmetric band -> tridiagonal (the reduction for the symmetric eigenvalue
 * problem, which the paper names as the sister use of bulge chasing; its own
 * method is the non-symmetric band -> bidiagonal one).  The same successive
 * band reduction and step geometry (Sec. III, Algorithm 1), with one Householder
 * reflector per step applied from both sides (A <- H A H).  T = Q^T A Q with Q
 * orthogonal, Q e1 = e1; eigenvalues are preserved.
 *   band     device pointer, LAPACK LOWER band of `dtype`: A(i, j) =
 *            band[(i - j) + j * ldband] for 0 <= i - j <= b, ldband >= b + 1
 *            (the symmetric A's lower triangle; rows past n - 1 are ignored).
 *   d, e     device pointers to n and max(n - 1, 0) doubles: the diagonal and
 *            sub-diagonal of T.
 *   dtype    BB_F64 or BB_F32 storage (reflectors in FP64); BB_F16 returns
 *            BB_ERR_UNSUPPORTED.  Tilewidths 1..32 (bb_set_params' tw; default 32);
 *            bb_set_params' groups_per_cu and lag apply, the other fields do not.
 * Argument numbers as bb_reduce.  Working memory is stream-ordered and freed by
 * the call.  FP64 results are bitwise independent of the launch shape.
 */
int bb_sym_reduce(int64_t n, int64_t b, bb_dtype_t dtype, const void *band, int64_t ldband,
                  double *d, double *e, void *stream);

/* Smallest safe step lag of the symmetric chase for a stage leaving bandwidth c
 * (c >= 1): 2, or 3 when c = 1. */
int bb_sym_min_lag(int64_t c);

/* Algorithmic bytes of the symmetric chase: read + write of the lower-triangle
 * entries every step touches (column k's segment, the left-pass columns, the
 * diagonal block's lower triangle, the right-pass rows), summed over all steps. */
double bb_sym_model_bytes(int64_t n, int64_t b, int elem_size, int tw);

/*
 * Reduce `count` independent bands of uneven n_i, b_i in one persistent launch
 * that draws (matrix, stage, sweep) tasks from a device work queue.  The paper
 * has no batched form: this entry point is this library's addition; each
 * matrix undergoes exactly the reduction of bb_reduce (Sec. III, Algorithm 1).  All host
 * arrays have `count` entries; band[i], d[i], e[i] are device pointers as in
 * bb_reduce.  Argument numbers: count=1, n=2, b=3, dtype=4, band=5, ldband=6,
 * d=7, e=8.  A matrix with an invalid entry makes the whole call fail with
 * the argument number of the array, before any work is enqueued.
 * The first call for a given (count, n[], b[], dtype, parameters, stream)
 * builds a plan and allocates its device workspace (hipMalloc); later calls
 * with the same key reuse it and allocate nothing, so they may be captured
 * into a hipGraph (the captured copy of the pointer arrays reads them from a
 * pinned host buffer kept for captures at replay time: replays use the
 * pointers of the most recent CAPTURED call with that key; direct calls stage
 * theirs in a separate buffer).  Calls sharing a plan must not overlap in
 * time; bb_release() frees all plans.
 */
int bb_reduce_batched(int64_t count, const int64_t *n, const int64_t *b, bb_dtype_t dtype,
                      const void *const *band, const int64_t *ldband,
                      double *const *d, double *const *e, void *stream);

/*
 * Singular values of the upper bidiagonal B = bidiag(d, e) that bb_reduce
 * returns (the paper computes them on the CPU, Sec. V-A; this is the on-device
 * alternative).  sigma(B) are the non-negative eigenvalues of the 2n x 2n
 * Golub-Kahan tridiagonal (zero diagonal, off-diagonal d0, e0, d1, ..., d_{n-1});
 * a group of four threads finds each by multisection on the Sturm count of
 * that matrix (the signs of its leading minors, on B scaled by a power of two),
 * to an absolute accuracy of about 4 eps sigma_i + 2^-60 ||B||.
 *   n        order (0 <= n <= 2^29).
 *   d, e     device pointers to n and max(n - 1, 0) doubles (e may be NULL if n <= 1).
 *   sigma    device pointer to n doubles: sigma_0 >= sigma_1 >= ... >= 0 (output).
 *   stream   hipStream_t.  Asynchronous; allocates nothing.
 * Argument numbers for -i: n=1, d=2, e=3, sigma=4.  A NaN or infinite entry
 * makes every output NaN.
 */
int bb_bidiag_sigma(int64_t n, const double *d, const double *e, double *sigma, void *stream);

/* Set (p != NULL) or reset to automatic (p == NULL) the process-wide tuning
 * parameters; invalid values are rejected with -1 and leave the state unchanged. */
int bb_set_params(const bb_params_t *p);
/* Read the current process-wide parameters (0 fields = automatic). */
int bb_get_params(bb_params_t *p);

/*
 * Autotune for one problem shape.  The paper tunes its three knobs (threads per
 * block, inner tilewidth, maximum blocks; Sec. III-C and the hyper-parameter
 * study of Sec. V) by brute-force search and names automatic tuning as future
 * work (Sec. VII); this is that search, ranked by a model and judged by time.
 * A short list of parameter sets (the built-in
 * defaults and shapes that win in other regimes; fields fixed by bb_set_params
 * are kept in all of them) is ranked by a critical-path model; the defaults and
 * the best five others are each timed three times (after one untimed run) on a
 * synthetic band of this shape (n capped at 32768) on `stream`, the median
 * decides, and the winner -- the defaults unless another set is at least 1 %
 * faster -- is cached for (floor(log2 n), min(b, n-1), dtype).  Later calls of
 * bb_reduce for that key use the cached fields that bb_set_params leaves at 0.
 * *out (may be NULL) receives the first-stage launch shape of the winner.
 * Allocates stream-ordered device memory and synchronises `stream`.
 * bb_release() clears the cache.
 */
int bb_autotune(int64_t n, int64_t b, bb_dtype_t dtype, void *stream, bb_params_t *out);

/*
 * Autotune the batched form for one exact batch (count, n[], b[], dtype; host
 * arrays as in bb_reduce_batched).  The same search as bb_autotune (Sec. III-C
 * knobs, Sec. VII's automatic tuning), over the batched form's candidates
 * (workgroups per CU, tilewidth, threads per window, sweeps per group): each is
 * timed three times on synthetic bands of exactly these shapes and the median
 * decides; the defaults stay unless a candidate is at least 1 % faster.  The
 * winner is cached for this exact batch and used by later bb_reduce_batched
 * calls with the same (count, n[], b[], dtype) for the fields bb_set_params
 * leaves at 0.  The winner's batch plan (and its workspace) is kept, so the next
 * call with the batch allocates nothing and may be captured into a hipGraph.
 * *out (may be NULL) receives the winner's launch shape.  Allocates stream-ordered
 * device memory and synchronises `stream`.  Argument numbers: count=1, n=2, b=3,
 * dtype=4.  bb_release() clears the cache.
 */
int bb_autotune_batched(int64_t count, const int64_t *n, const int64_t *b, bb_dtype_t dtype,
                        void *stream, bb_params_t *out);

/* The parameters (first-stage launch shape) bb_reduce would use for this shape
 * now: bb_set_params fields, then an autotuned entry, then the defaults.  Host
 * only; no device work.  -4 if out is NULL. */
int bb_resolved_params(int64_t n, int64_t b, bb_dtype_t dtype, bb_params_t *out);

/* Device bytes of working memory one bb_reduce call of this shape allocates: the
 * working band of b + 2 TW + 1 rows per column (the band height given in the
 * storage paragraph of Sec. IV) plus the dependency counters.  Not in the paper;
 * a sizing query of this library.  0 for n <= 0 or b < 0. */
size_t bb_workspace_bytes(int64_t n, int64_t b, bb_dtype_t dtype);

/*
 * Algorithmic bytes of the reduction: the read + write of every window a step
 * touches (the L-shaped union of the right reflector's row block and the left
 * reflector's column block), summed over every step of every stage, for an
 * element of `elem_size` bytes under inner tilewidth `tw`.
 */
double bb_model_bytes(int64_t n, int64_t b, int elem_size, int tw);

/*
 * Stage plan for bandwidth b under inner tilewidth tw (host only): fills up to
 * `max_stages` entries of bs (bandwidth entering the stage), tws (tilewidth),
 * cs (bandwidth left) and lags (half-step lag used between sweeps); returns
 * the number of stages, or a negative argument error.
 */
int bb_plan(int64_t b, int tw, int max_stages, int *bs, int *tws, int *cs, int *lags);

/* Smallest safe half-step lag for a stage that leaves bandwidth c (c >= 1). */
int bb_min_lag(int64_t c);

/* Synchronise `stream` and return (and clear) the error word of the current
 * device: BB_OK or BB_ERR_TIMEOUT, or BB_ERR_HIP if the synchronisation failed.
 * The error word is kept per DEVICE, not per stream: a watchdog timeout raised
 * by a call on another stream of the same device is reported (and cleared) by
 * whichever bb_stream_status call reads it first. */
int bb_stream_status(void *stream);

/*
 * Kernel timing (diagnostics for benchmarks).  While enabled, every bb_reduce
 * call records a hipEvent pair on its stream around each launch of the stage
 * (bulge-chasing) kernel.  bb_timing_read synchronises on those events, returns
 * the summed milliseconds and the number of launches since the previous read
 * (either pointer may be NULL) and forgets them.  Disabled by default.
 */
int bb_timing_enable(int on);
int bb_timing_read(double *stage_ms, int64_t *stage_launches);

/* Free cached host/device resources of the library (pools, autotune cache). */
int bb_release(void);

/* Static text for an error code (negative codes: "invalid argument"). */
const char *bb_error_string(int code);

#ifdef __cplusplus
}
#endif

#endif /* BB_H */
