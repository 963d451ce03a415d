/*
 * spamm.h -- C ABI of the MI355X (gfx950) SpAMM / Newton-Schulz library.
 *
 * Implements the Sparse Approximate Matrix Multiply a (x)_tau b of
 * Challacombe, Haut & Bock, "A N-Body Solver for Square Root Iteration"
 * (Sec. 2, eq. "newspamm", error bound of Sec. 2.1) and the dual-channel
 * coupled Newton-Schulz iteration for s^{1/2} and s^{-1/2} built on it
 * (Sec. 3.2, eq. "cannonical").
 *
 * Conventions shared by every entry point:
 *   - Matrix arguments are DEVICE pointers owned by the caller: square, FP64,
 *     row-major with leading dimension ld >= n.  The library never frees or
 *     retains them past the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *     stream).  Work is enqueued on it; every entry point that returns host
 *     values (statistics, results, statuses) synchronises that stream before
 *     returning, so outputs are complete when the call returns.
 *   - Return value: a spamm_status.  0 = success; > 0 = warning with valid
 *     outputs; < 0 = error, outputs undefined, text in spamm_last_error().
 *   - Invalid arguments (n <= 0, ld < n, tau < 0 or NaN, tol <= 0, maxit < 0,
 *     leaf not in {16, 32, 64}, an unknown precision, a NULL required pointer)
 *     return SPAMM_EINVAL before any work is enqueued.
 *   - A context owns all scratch memory (tiles, norm pyramids, task lists).
 *     Use one context per host thread; calls on one context are not
 *     thread-safe.  Scratch grows on demand and is reused across calls.
 *   - Leaf block order: the paper's N_b; n need not be a multiple of it
 *     (zero padding, outside the logical identity).
 */
#ifndef SPAMM_H
#define SPAMM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPAMM_OK = 0,
    SPAMM_NOT_CONVERGED = 1, /* maxit updates done without r < tol; outputs = last iterate     */
    SPAMM_STAGNATED = 2,     /* opt-in stagnation stop fired; outputs = last iterate           */
    SPAMM_EINVAL = -1,       /* invalid argument or input (NaN/Inf, asymmetric s)              */
    SPAMM_ENOMEM = -2,       /* device or pinned allocation failed                             */
    SPAMM_EDIVERGED = -3,    /* r_k not finite or r_k > 10 max(r_0, sqrt(n))                   */
    SPAMM_EHIP = -4,         /* a HIP runtime call failed                                      */
    SPAMM_ECAPACITY = -5     /* caller's triple buffer too small (stats still filled)          */
} spamm_status;

/* Arithmetic of the leaf products.  Norms, the cull decision, the Newton-
 * Schulz residual and trace are FP64 in every mode; norms are taken of the
 * values as stored in the leaf precision. */
typedef enum {
    SPAMM_F64 = 0,    /* FP64 tiles, FP64 MFMA                                       */
    SPAMM_F32 = 1,    /* FP32 tiles, FP32 MFMA, FP32 accumulation                    */
    SPAMM_BF16X3 = 2, /* FP32 tiles; each product a_hi b_hi + a_hi b_lo + a_lo b_hi
                         on BF16 MFMA with FP32 accumulation (a = a_hi + a_lo, two
                         bf16 pieces: O(2^-16) relative error per product)          */
    SPAMM_BF16X6 = 3  /* FP32 tiles split into three bf16 pieces a = a_hi + a_mid + a_lo
                         (exact for every FP32 value); the product of two 32-k
                         slices is the six terms down to 2^-16 relative (a_lo b_hi,
                         a_hi b_lo, a_mid b_mid, a_mid b_hi, a_hi b_mid, a_hi b_hi,
                         in that order) on BF16 MFMA summed in FP32, and the slice
                         sums are accumulated in FP64: FP32 storage is the error */
} spamm_prec;

typedef struct spamm_ctx spamm_ctx;

/* Create a context on HIP device `device` (made current for the calls made
 * through this context).  *ctx receives the handle.  Errors: EINVAL (NULL
 * ctx or bad device), EHIP. */
int spamm_create(spamm_ctx **ctx, int device);

/* Release the context and all its device memory, pooled memory and solves
 * begun and not finished included (synchronises the device). */
int spamm_destroy(spamm_ctx *ctx);

/* Thread-local text describing the most recent status < 0 on this thread. */
const char *spamm_last_error(void);

/* Number of entries of a norm pyramid for order n and leaf b:
 * (4^(L+1) - 1)/3 with L = ceil(log2(ceil(n/b))).  Returns -1 on bad args. */
int64_t spamm_pyramid_len(int64_t n, int leaf);

/*
 * Frobenius-norm quadtree of A (Sec. 1, quadtree norm equation): the squared
 * norm of a node is the sum of its four children's squared norms, summed as
 * (q00 + q01) + (q10 + q11); leaves are the b x b blocks.
 *
 * pyramid: DEVICE, spamm_pyramid_len(n, leaf) doubles, receives NORMS (square
 *   roots), leaves first: the leaf level is 2^L x 2^L row-major (blocks past
 *   ceil(n/b), the virtual blocks of the padded tree, are 0), then each parent
 *   level up to the root (one value).
 * root_norm_host: optional HOST double, receives ||A||_F (synchronises).
 */
int spamm_norms(spamm_ctx *ctx, const double *A, int64_t n, int64_t ld, int leaf, double *pyramid,
                double *root_norm_host, void *stream);

typedef struct {
    int64_t retained; /* |R|, retained leaf triples                          */
    int64_t possible; /* ceil(n/b)^3                                         */
    double thr;       /* tau * (||A|| * ||B||)                               */
    double flops;     /* 2 b^3 |R|                                           */
} spamm_stats;

/*
 * C = A (x)_tau B (Sec. 2, eq. "newspamm"): every leaf triple (i,j,k) with
 * ||A_ik|| * ||B_kj|| < tau * (||A|| * ||B||) is culled (strict <, so tau = 0
 * keeps all and is the dense product); each C block accumulates its retained
 * k in increasing order.  The retained set equals the paper's recursive one
 * because parent norms bound child norms.  ||C - A B||_F <= n^2 tau ||A|| ||B||
 * (Sec. 2.1).
 *
 * A, B: DEVICE inputs; C: DEVICE output (n x n, same ld; may not alias A/B).
 * prec: a spamm_prec.  triples: optional DEVICE int32[cap][3] receiving the
 *   retained (i,j,k) sorted lexicographically; SPAMM_ECAPACITY if |R| > cap
 *   (C and stats are still valid).  stats: optional HOST output.
 * Synchronises the stream when stats or triples are requested.
 */
int spamm_multiply(spamm_ctx *ctx, const double *A, const double *B, double *C, int64_t n, int64_t ld,
                   double tau, int leaf, int prec, int32_t *triples, int64_t cap, spamm_stats *stats,
                   void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * product as spamm_multiply, C = A (x)_tau B, with the same kernels and so
 * the same results, that allocates nothing.  Every working buffer (tiles,
 * norm pyramids, task list, product table) is carved from a static device
 * array of SPAMM_NOALLOC_BYTES per GPU, located when a context is created on
 * that GPU and held until the process ends.
 *
 * A, B: DEVICE inputs; C: DEVICE output (n x n, leading dimension ld >= n;
 *   C may not alias A or B).  tau, leaf, prec as spamm_multiply.
 * No statistics or triples, and no synchronisation: the work is enqueued on
 * `stream` and the call returns.
 * Errors: EINVAL for invalid arguments and for sizes whose buffers exceed
 *   the static array (about n <= 1100 for FP64 tiles, n <= 1500 for FP32 and
 *   BF16x3 tiles; the message names the bytes needed); EHIP.
 * Every call on one GPU shares that GPU's array, which keeps the last call's
 * contents (what must start at zero is cleared by the call): calls that
 * overlap on one GPU (other streams, other host threads) race and must be
 * serialised by the caller.
 */
#define SPAMM_NOALLOC_BYTES 33554432u /* 32 MiB */
int spamm_multiply_noalloc(spamm_ctx *ctx, const double *A, const double *B, double *C, int64_t n, int64_t ld,
                           double tau, int leaf, int prec, void *stream);

typedef struct {
    int leaf;            /* N_b in {16, 32, 64}; 0 = 32                                    */
    int prec;            /* spamm_prec                                                     */
    double tau_s;        /* threshold of the y channel h (x) y; < 0 = tau (Sec. 4.1)         */
    double mu_rel;       /* Tikhonov shift s + mu_rel * c0 * I, c0 the Gershgorin bound of s
                            (Sec. 6); 0 = none                                             */
    int stagnation_stop; /* 1 = stop when r_k >= 0.99 r_best, r_best = min(r_0..r_{k-1}),
                            twice in a row while r_best < 1/2 or n |t_k| < 1/2 (then every
                            eigenvalue of an exact iterate is within 1/2 of 1, where an
                            update shrinks r more than 2x: no 1% gain means the
                            tau/rounding floor)                                         */
    int damped;          /* 1 = the damped map of Sec. 4.2 "Mapping": h = (sqrt(a)/2)
                            (3 I - a xs), xs = e I + (1 - 2e) x, with the scaling
                            a(t) = 1 + 1.85/(1 + exp(-50 (t - 0.35))) and stabilisation
                            e(t) = 0.1/(1 + exp(-75 (t - 0.30))) of the trace error
                            t_k = (n - tr x_k)/n; both switched off (a = 1, e = 0) once
                            t_k < 0.1, so the fixed point stays x = I.  0 = the plain
                            map h = 1.5 I - 0.5 x                                       */
    int single;          /* 1 = the single-channel instance (Sec. 3.2, eq. "single";
                            the implicit y channel as described in Sec. 5.3):
                            z_0 = I_n; y_k = s' (x)_{tau_s} z_k (the y channel implicit in
                            the product with s, taken rightmost at the tighter tau_s),
                            x_k = z_k^T (x)_tau y_k, z_{k+1} = z_k (x)_tau h_k; Y = sqrt(c)
                            y_k.  Same stop tests and map.  0 = dual channel            */
} spamm_ns_opts;

typedef struct {
    int iterations;        /* updates performed                                         */
    double resid;          /* last in-loop r_k = ||I_n - y_k (x)_tau z_k||_F             */
    double trace_err;      /* last t_k = (n - tr x_k)/n (Sec. 4.2)                       */
    double scale;          /* c, the Gershgorin bound used to scale s                    */
    int64_t triples_total; /* sum of |R| over all products                               */
    double flops_total;    /* 2 b^3 triples_total                                        */
} spamm_ns_result;

/*
 * Dual-channel coupled Newton-Schulz (Sec. 3.2, eq. "cannonical") with the map
 * h[x] = (3 I - x)/2.  s' = (s + mu I)/c with c = max_i sum_j |s_ij| (a bound
 * on the largest eigenvalue, so the spectrum lies in (0, 1]); y_0 = s',
 * z_0 = I_n.  For k = 0, 1, ...: x_k = y_k (x)_tau z_k; r_k = ||I_n - x_k||_F;
 * stop with OK when r_k < tol, EDIVERGED when r_k is not finite or exceeds
 * 10 max(r_0, sqrt(n)), STAGNATED (opt-in) after two consecutive
 * r_k >= 0.99 r_best (r_best = min(r_0..r_{k-1})) while r_best < 1/2 or
 * n |t_k| < 1/2, NOT_CONVERGED when k == maxit; otherwise
 * h_k = 1.5 I_n - 0.5 x_k, y_{k+1} = h_k (x)_{tau_s} y_k, z_{k+1} = z_k (x)_tau h_k.
 *
 * s: DEVICE input, symmetric (max|s - s^T| <= 1e-14 max|s|) and finite, else
 *   EINVAL.  Y ~ s^{1/2} = sqrt(c) y_k and Z ~ s^{-1/2} = z_k / sqrt(c):
 *   DEVICE outputs with leading dimension ld.  opts: NULL = defaults (leaf 32,
 *   F64, tau_s = tau, no shift, literal stop rule).  res: optional HOST output.
 * The stop test runs on the device; the host reads the solve's state back once
 * per step of up to four iterations (iterations after a stop do no work) and
 * synchronises at the end.
 */
int ns_sqrt(spamm_ctx *ctx, const double *s, double *Y, double *Z, int64_t n, int64_t ld, double tau,
            double tol, int maxit, const spamm_ns_opts *opts, spamm_ns_result *res, void *stream);

/*
 * Step API: the same iteration as ns_sqrt, advanced explicitly so
 * that many solves share launches (batched solves of uneven n) and solves
 * can join and leave between steps (continuous batching for serving).
 * ns_sqrt is spamm_solve_begin + spamm_solve_step until done +
 * spamm_solve_finish, so results are identical whichever way a solve runs.
 */
typedef struct spamm_solve spamm_solve;

/* Device bytes one solve holds from begin to finish (for admission control):
 * five b x b-tiled iterates (dual: y, y', z, z', h; single: s', y_k, z, z',
 * h, and a sixth, z^T) in the leaf precision, as many norm pyramids, three
 * task lists of ceil(n/b)^3 int32, per-tile partials and the per-iteration
 * records.  single: 0 = dual channel, 1 = single channel.  0 on bad
 * arguments. */
size_t spamm_solve_footprint(int64_t n, int leaf, int prec, int maxit, int single);

/* Checks s (as ns_sqrt), scales it, takes the solve's device memory from the
 * context's pool (a block of at most 1.25 times the footprint plus 16 MiB;
 * allocating only when no pooled block fits) and sets
 * y_0 = s', z_0 = I_n.  It also reserves in the pool the tables and pinned
 * read-back buffer of a step over every unfinished solve of its (precision,
 * leaf, channel) group on this context, so steps and finishes need no
 * allocation.  s may be freed once this returns (synchronises).  *out
 * receives the solve; errors as ns_sqrt (EINVAL, ENOMEM, EHIP). */
int spamm_solve_begin(spamm_ctx *ctx, const double *s, int64_t n, int64_t ld, double tau, double tol, int maxit,
                      const spamm_ns_opts *opts, spamm_solve **out, void *stream);

/* Advances every running solve in solves[0..count) by `iterations` (>= 1)
 * iterations: each iteration of all of them is one shared sequence of
 * launches per (precision, leaf, channel) group; the stop tests run on the
 * device.  The groups run concurrently on streams of the context that start
 * after the work already on `stream`, and `stream` waits for all of them.
 * Stopped solves in the list do no work; a solve may appear once.  The
 * tables and captured graph of a group are rebuilt only when its list of
 * unfinished solves changes (a solve joins or is finished), from memory
 * reserved by spamm_solve_begin.  Synchronises once.  Returns the number of
 * solves of the list still running, or < 0 on error (EINVAL for a NULL,
 * repeated or foreign solve). */
int spamm_solve_step(spamm_ctx *ctx, spamm_solve *const *solves, int count, int iterations, void *stream);

/* Host-side state after the last step: *done = 1 once stopped; res as for
 * ns_sqrt.  Returns SPAMM_OK while running, else the solve's final status. */
int spamm_solve_poll(spamm_solve *solve, int *done, spamm_ns_result *res);

/* Writes Y = sqrt(c) y_k and Z = z_k / sqrt(c) (either may be NULL), records
 * the solve's history for spamm_ns_history, releases the solve (its device
 * memory and its tables go back to the context's pool, nothing is freed) and
 * returns its status (NOT_CONVERGED if it was still running).  Synchronises. */
int spamm_solve_finish(spamm_ctx *ctx, spamm_solve *solve, double *Y, double *Z, int64_t ld, void *stream);

/* Retained (i, j, k) leaf triples of the most recent product of one channel
 * of a solve (the "vol" of Secs. 5.4 and 6.2 and the ijk volumes shown for lensing,
 * Sec. 7.2): which = 0 the x product, 1 the y product, 2 the z product.
 * After a step the x product is that of the last iteration performed; the
 * y and z products are those of the last update (in the single instance the
 * y product is y_k of the last iteration).  triples: DEVICE int32[cap][3],
 * sorted by (i, j, k); *count (HOST, optional) receives |R|; ECAPACITY (and
 * the count) when |R| > cap.  Synchronises the stream. */
int spamm_solve_triples(spamm_ctx *ctx, spamm_solve *solve, int which, int32_t *triples, int64_t cap,
                        int64_t *count, void *stream);

/*
 * Product representation of the regularised inverse factor (Sec. 6.1) by
 * iterative regularisation (Sec. 6.3).  Slice 0: W = (s + mu_0 c0 I)^{-1/2}
 * by ns_sqrt at the slice threshold (c0 the Gershgorin bound of s).  Then for
 * each finer shift mu_j: the residual congruence M_j = W^T (x)_{tau_r}
 * ((s + mu_j c0 I) (x)_{tau_r} W), through its symmetric part (symmetric in
 * exact arithmetic); Z_j = M_j^{-1/2} by ns_sqrt at the slice threshold; and
 * W <- W (x)_{tau_r} Z_j, so that W^T (s + mu_j c0 I) W -> I.  The new slice
 * multiplies on the right, the order under which that congruence holds (the
 * paper prints the reverse order, equal in exact arithmetic).
 */
#define SPAMM_MAX_SLICES 16
typedef struct {
    int leaf;               /* N_b of every product and solve; 0 = 32                      */
    int prec;               /* spamm_prec of every product and solve                       */
    int nslices;            /* 1 .. SPAMM_MAX_SLICES                                       */
    const double *mu_rel;   /* HOST, nslices shifts relative to c0, each >= 0 (decreasing)  */
    double tau_slice;       /* tau of each slice's Newton-Schulz solve                      */
    double tau_s_slice;     /* its tau_s; < 0 = tau_slice                                    */
    double tau_r;           /* tau of the residual congruences and of the slice products    */
    double tol;             /* each slice's stop tolerance                                   */
    int maxit;              /* each slice's update limit                                     */
    int stagnation_stop;    /* as spamm_ns_opts                                              */
    int damped;             /* as spamm_ns_opts                                              */
} spamm_prodrep_opts;

typedef struct {
    int nslices_done;                    /* slices computed (stops at a failing slice)   */
    int status[SPAMM_MAX_SLICES];        /* each slice's ns_sqrt status                  */
    int iterations[SPAMM_MAX_SLICES];    /* each slice's update count                    */
} spamm_prodrep_result;

/* s: DEVICE, symmetric (as ns_sqrt); W: DEVICE output, row-major with
 * leading dimension ld >= n.  Working memory (six n x ld FP64 matrices) is
 * allocated for the call and freed before it returns.  Returns the first
 * negative slice status (EDIVERGED: W holds the last good factor), EINVAL,
 * ENOMEM, EHIP, else OK.  res: optional HOST output.  Synchronises. */
int spamm_product_rep(spamm_ctx *ctx, const double *s, double *W, int64_t n, int64_t ld,
                      const spamm_prodrep_opts *opts, spamm_prodrep_result *res, void *stream);

/* Per-iteration record of the most recent finished solve on this context, HOST
 * outputs of capacity cap entries: r[k], t[k] and nR[3k..3k+2] = |R| of x_k,
 * y_{k+1}, z_{k+1} (the last two are 0 where no update followed).  Returns the
 * number of entries available (iterations + 1), or < 0 on error. */
int spamm_ns_history(spamm_ctx *ctx, double *r, double *t, int64_t *nR, int cap);

/* Whether spamm_solve_step (and so ns_sqrt) replays each solve set's
 * iteration as a captured HIP graph (default 1).  The graph is captured on the
 * set's second step (its first step launches plainly, so sets that last one
 * step cost no capture), on a stream the context owns, ordered after the
 * caller's stream by an event, and the caller's stream is ordered after it;
 * steps block the host either way.  While launch timing is enabled, plain
 * launches are used. */
int spamm_set_graphs(spamm_ctx *ctx, int enable);

/* Launch timing, for measurement.  While enabled, every leaf-product launch
 * (kind 0), cull launch (kind 1) and norm-pyramid launch (kind 2) enqueued
 * through this context is bracketed by a pair of HIP events recorded on the
 * same stream.  For product tables of at most 1024 tiles the cull launch also
 * orders the work and writes the job list, and with the plain map the
 * pyramid of such a solve's x product is built inside the (untimed) stop
 * decision.  Events come from a fixed pool created at enable time (no
 * allocation while solving); when it is exhausted recording stops silently.
 * spamm_profile_enable(ctx, 1) also clears earlier records; 0 disables. */
int spamm_profile_enable(spamm_ctx *ctx, int enable);

/* Durations in milliseconds of the recorded launches of `kind`, in launch
 * order, into HOST ms[cap].  Returns the number recorded (may exceed cap), or
 * < 0 on error.  The recorded work must be complete (every entry point that
 * reports results has synchronised its stream).  Clears nothing. */
int spamm_profile_read(spamm_ctx *ctx, int kind, double *ms, int cap);

/* Forget the recorded launches (the pool is reused). */
int spamm_profile_reset(spamm_ctx *ctx);

/* Device and pinned host allocations this context has made so far: scratch
 * growth, solve arenas, plan tables and read-back buffers.  Memory of
 * finished solves and dropped tables is pooled and reused, not freed, so a
 * warm context steps and finishes solves without adding to this count.
 * Returns -1 for a NULL context. */
int64_t spamm_alloc_count(spamm_ctx *ctx);

/* Largest number of device bytes the context keeps pooled (free solve arenas
 * and plan tables; default: no limit).  Memory that a finishing solve or a
 * dropped plan returns beyond it is freed at once, which synchronises the
 * device; memory pooled beyond a new limit is freed now.  For callers that
 * share the device with other allocations (a server sizing its admission
 * budget).  Errors: EINVAL (NULL ctx), EHIP. */
int spamm_set_pool_limit(spamm_ctx *ctx, size_t bytes);

#ifdef __cplusplus
}
#endif

#endif /* SPAMM_H */
