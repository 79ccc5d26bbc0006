/*
 * pogs.h - C ABI of a graph-form ADMM solver for MI355X (gfx950).
 *
 * Solves   minimize f(y) + g(x)   subject to   y = A x          (Section 1)
 * with A dense (m x n) and f, g separable, each term in the parametric form
 * of Section 5:
 *     f_i(y) = c_i h_i(a_i y - b_i) + d_i y + (e_i / 2) y^2,   c_i >= 0, e_i >= 0.
 *
 * The method is graph projection splitting (Section 3.1, Algorithm 1) with
 * over-relaxation (Section 3.2), residual stopping on the half-step tuple
 * (Sections 3.3-3.4), diagonal pre-conditioning by regularised
 * Sinkhorn-Knopp equilibration plus Frobenius normalisation (Sections 4.1,
 * 4.2, Algorithm 2, Section 5) and the adaptive penalty of Section 4.3
 * (Algorithm 3).  The graph projection uses the reduced update of Section 3.5
 * with a factorisation of I + A^T A (m >= n) or I + A A^T (m < n) computed
 * once per matrix and cached in the context.
 *
 * Conventions for every entry point:
 *   - return value: 0 (POGS_OK) or a negative POGS_E* code; nothing is
 *     launched when an argument check fails.  Failing to converge is not an
 *     error: it is reported in pogs_result.status.
 *   - pointers tagged POGS_HOST are host memory, POGS_DEVICE are device
 *     memory on the current HIP device.  Input buffers are only read and may
 *     be freed by the caller as soon as the call returns (the library copies
 *     what it keeps).  Output buffers are caller-allocated.
 *   - "stream" arguments are a hipStream_t passed as void*; NULL means the
 *     library's own stream (one per calling thread and device, created on
 *     first use and kept until the process ends; non-blocking, so it is not
 *     ordered after work on the legacy null stream).  Calls are synchronous
 *     with respect to the host:
 *     they return after their device work has finished.
 *   - A context (pogs_ctx) is not thread-safe; use one per thread.  The batch
 *     engine (pogs_batch) is thread-safe.
 */
#ifndef POGS_H
#define POGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define POGS_OK            0
#define POGS_EINVAL       -1   /* bad argument (size, pointer, non-finite data,
                                  c < 0 or e < 0, a == 0 with c > 0, unknown h) */
#define POGS_ENOMEM       -2   /* device or host allocation failed */
#define POGS_EDEVICE      -3   /* a HIP runtime call failed */
#define POGS_EAGAIN       -4   /* batch: request can never fit the memory budget,
                                  or the queue is full */
#define POGS_ENOTFOUND    -5   /* batch: unknown ticket */
#define POGS_EUNSUPPORTED -6   /* valid request the library does not implement */
#define POGS_ETOOBIG      -7   /* input larger than the fixed device buffer of an
                                  allocation-free entry point */

/* ---- solve status (pogs_result.status) ---------------------------------- */
#define POGS_CONVERGED  0      /* r_pri < eps_pri and r_dual < eps_dual */
#define POGS_MAXITER    1      /* iteration cap reached */
#define POGS_NUMERICAL  2      /* a residual became non-finite */
#define POGS_CANCELLED  3      /* batch: cancelled before completion */
#define POGS_FAILED     4      /* batch: the request could not be set up on the
                                  device; pogs_result.error holds the code
                                  (POGS_ENOMEM, POGS_EDEVICE, or POGS_EINVAL for
                                  non-finite entries found on the device) */

typedef enum { POGS_F32 = 0, POGS_F64 = 1 } pogs_dtype;
typedef enum { POGS_ROW_MAJOR = 0, POGS_COL_MAJOR = 1 } pogs_order;
typedef enum { POGS_HOST = 0, POGS_DEVICE = 1 } pogs_mem;

/* Base functions h of the parametric form (Section 5). */
typedef enum {
  POGS_H_ZERO = 0,      /* 0 */
  POGS_H_IDENTITY = 1,  /* u */
  POGS_H_ABS = 2,       /* |u| */
  POGS_H_SQUARE = 3,    /* u^2 / 2 */
  POGS_H_HUBER = 4,     /* u^2/2 for |u| <= 1, |u| - 1/2 otherwise */
  POGS_H_HINGE = 5,     /* max(0, u) */
  POGS_H_LOGISTIC = 6,  /* log(1 + e^u) */
  POGS_H_IND_GE0 = 7,   /* indicator of u >= 0 */
  POGS_H_IND_LE0 = 8,   /* indicator of u <= 0 */
  POGS_H_IND_EQ0 = 9,   /* indicator of u == 0 */
  POGS_H_IND_BOX01 = 10, /* indicator of 0 <= u <= 1 */
  POGS_H_EXP = 11,       /* e^u */
  POGS_H_NEG_ENTR = 12,  /* u log u on u >= 0 (0 at 0), +inf for u < 0 */
  POGS_H_NEG_LOG = 13,   /* -log u on u > 0, +inf otherwise */
  POGS_H_RECIPR = 14,    /* 1/u on u > 0, +inf otherwise */
  POGS_H_MAX_NEG0 = 15   /* max(0, -u) */
} pogs_h;

/* A separable function of length len, in host memory.  Each of h, a..e is
 * either an array of len entries (stride 1) or a single entry used for every
 * element (stride 0).  A NULL parameter pointer means its default
 * (a = 1, b = 0, c = 1, d = 0, e = 0); h may not be NULL. */
typedef struct {
  int64_t len;
  int64_t stride;                 /* 1: per element, 0: broadcast entry 0 */
  const uint8_t *h;               /* pogs_h codes */
  const double *a, *b, *c, *d, *e;
} pogs_fn;

/* How the projection onto {(x, y) : y = A x} is computed (Section 3.5).
 * DIRECT: the reduced update with the inverse of I + A^T A (m >= n) or
 * I + A A^T (m < n), formed once at pogs_init from a float64 Cholesky factor.
 * CGLS: conjugate gradients on the least-squares form of the projection,
 * min ||x - c||^2 + ||A x - d||^2, started from the half step x_h and stopped
 * when its normal residual s = A^T (d - A x) + c - x has
 * rho ||s|| <= cg_tol * eps_dual (this iteration's dual tolerance) or after
 * cg_max_iter steps; no Gram matrix or factor is formed, so any min(m, n)
 * fits.  Each step reads A twice. */
typedef enum { POGS_PROJ_DIRECT = 0, POGS_PROJ_CGLS = 1 } pogs_projection;

/* Stopping rule (Section 3.4).  RESIDUAL: stop when ||A x_h - y_h|| < eps_pri
 * and ||A^T nu_h + mu_h|| < eps_dual; the half-step tuple is returned.  GAP:
 * stop when the gap eta = f(y) + g(x) + f*(nu) + g*(mu) of the primal and dual
 * feasible tuple the projection leaves, (x, y, mu, nu) = (x, A x, -rho x~,
 * -rho y~), is below eps_abs + eps_rel |f(y) + g(x)|; that tuple is returned
 * and bounds its own suboptimality by eta.  eta is +inf whenever the tuple
 * violates a constraint of f or g or lies outside the domain of a conjugate
 * (indicators, hinge, logistic, ...), so the rule suits functions with full
 * domains (or e > 0); it is checked from the second iteration on, in the
 * scaled variables (the gap is invariant under the scaling).  GAP needs the
 * direct projection. */
typedef enum { POGS_STOP_RESIDUAL = 0, POGS_STOP_GAP = 1 } pogs_stop_rule;

/* Solver parameters; pogs_params_default fills the values of Section 5. */
typedef struct {
  double eps_abs;        /* absolute tolerance (Section 3.4), default 1e-4 */
  double eps_rel;        /* relative tolerance, default 1e-3 */
  int32_t max_iter;      /* iteration cap, default 10000 */
  double rho0;           /* initial penalty, default 1 */
  double alpha;          /* over-relaxation (Section 3.2), default 1.7 */
  double delta;          /* adaptive-rho factor (Algorithm 3), default 1.05 */
  double tau;            /* adaptive-rho spacing (Algorithm 3), default 0.8 */
  int32_t adaptive_rho;  /* 1 = Algorithm 3 on (default), 0 = fixed rho */
  int32_t equil_iters;   /* Sinkhorn-Knopp sweeps (Algorithm 2), default 10;
                            0 = no pre-conditioning (D = E = I) */
  double eps_cmp;        /* machine epsilon in gamma = (m+n) sqrt(eps_cmp);
                            <= 0 selects the epsilon of the matrix dtype */
  int32_t chunk_iters;   /* iterations per device launch sequence between
                            host checks of the stop flag, default 20 */
  int32_t verbose;       /* 0 silent, 1 per-chunk log on stderr */
  int32_t projection;    /* POGS_PROJ_DIRECT (default) or POGS_PROJ_CGLS */
  int32_t cg_max_iter;   /* CGLS steps per projection at most, 1..1000, default 10 */
  double cg_tol;         /* CGLS stops when rho ||s|| <= cg_tol * eps_dual, default 0.1 */
  int32_t stop_rule;     /* POGS_STOP_RESIDUAL (default) or POGS_STOP_GAP */
  int32_t autotune;      /* 1 (default): pogs_init times the load policy of the
                            passes over A (cached or non-temporal loads, for the
                            row passes and the column passes) on the projection
                            (pass 1, solve, pass 2) of the context's shape,
                            interleaved over four rounds, and keeps the fastest
                            if it beats the size rule's policy (that of
                            autotune = 0) by 2 %; the choice is cached per
                            (m, n, dtype) in the process and changes no result
                            bit.  0: a matrix above 192 MB streams, others cache. */
  int32_t sparse_segment; /* pogs_init_sparse only: columns of A^T per segment
                            of its segmented copy (the passes over A^T gather
                            from one segment's piece of an m-vector at a time);
                            0 (default): 1 MB of the paired vector per segment,
                            with at least two entries per row piece on average.
                            >= 0; results depend on it only through the
                            summation order. */
} pogs_params;

/* Result of a solve: the half-step tuple (x, y, mu, nu) of the last iteration,
 * in the original (unscaled) variables (Section 5).  x, y, mu, nu are
 * caller-allocated buffers of n, m, n, m elements of the context's dtype in
 * memory space `mem`; any of them may be NULL to skip that copy. */
typedef struct {
  void *x, *y, *mu, *nu;
  pogs_mem mem;
  double optval;     /* f(y) + g(x) at the returned tuple (parametric terms only;
                        indicator terms are zero there by construction) */
  double r_pri, r_dual, eps_pri, eps_dual;  /* last residuals (scaled space) */
  double rho;        /* final penalty */
  int32_t iters;     /* iterations run */
  int32_t status;    /* POGS_CONVERGED / POGS_MAXITER / POGS_NUMERICAL / POGS_CANCELLED /
                        POGS_FAILED */
  double ms_setup;   /* setup time of the context this solve used (ms) */
  double ms_solve;   /* wall time of this solve (ms) */
  int32_t cg_steps;  /* CGLS steps over all projections (0 for DIRECT) */
  int32_t error;     /* status POGS_FAILED: the POGS_E* code of the failure, else 0 */
  double gap;        /* stop_rule GAP: eta of the last tuple tested (NaN otherwise) */
  double eps_gap;    /* its tolerance eps_abs + eps_rel |f + g| (NaN otherwise) */
} pogs_result;

typedef struct pogs_ctx pogs_ctx;

/* Fill *p with the defaults above.  POGS_EINVAL if p is NULL. */
int pogs_params_default(pogs_params *p);

/* Create a context for matrix A (m x n, element type dt, storage order ord,
 * leading dimension lda >= n for row-major or >= m for column-major, in
 * memory `mem`).  Copies A to the device, converts it to row-major storage of
 * dt with a 64-element-aligned leading dimension, runs Algorithm 2
 * (params->equil_iters sweeps, p = 2, gamma = (m + n) sqrt(eps_cmp)), the
 * Frobenius normalisation of Section 4.1.2, scales A in place to D A E, and,
 * for params->projection == POGS_PROJ_DIRECT, forms the Gram matrix (Section
 * 3.5), factors I + G by Cholesky in float64 and keeps the inverse for later
 * solves (POGS_PROJ_CGLS skips the Gram matrix and the factor).  params may
 * be NULL (defaults).
 * Errors: EINVAL (m, n <= 0, NULL pointers, lda too small, non-finite A,
 * invalid params), EUNSUPPORTED (direct projection with min(m, n) > 32768),
 * ENOMEM, EDEVICE.  On error *out is set to NULL. */
int pogs_init(pogs_ctx **out, int64_t m, int64_t n, const void *A, pogs_dtype dt,
              pogs_order ord, int64_t lda, pogs_mem mem, const pogs_params *params,
              void *stream);

/* Create a context for a sparse A (m x n) in compressed rows: row i holds the
 * entries colind[rowptr[i] .. rowptr[i + 1]) (0-based column indices, any
 * order, repeated indices add up) with values val (dtype dt); rowptr has
 * m + 1 entries, rowptr[0] = 0 and rowptr[m] = nnz.  All three arrays in
 * memory `mem`, copied (the caller may free them on return).  The library
 * keeps A^ = D A E twice in compressed rows on the device, as A^ and as its
 * transpose (built by a stable counting sort over the columns), runs
 * Algorithm 2 and the Frobenius normalisation of Section 4.1.2 with row passes
 * over both, and projects by CGLS (Section 3.5, indirect; no factorisation of
 * a sparse K): solves on this context use POGS_PROJ_CGLS whatever
 * params->projection says, with cg_max_iter and cg_tol as given.  Warm starts
 * work as on a dense context (y = A^ x and x~ = -A^T y~ as row passes over
 * the two copies).  The gap rule, pogs_project and pogs_solve_path are not
 * available on it (EUNSUPPORTED).  Limits: nnz, m, n below 2^31 (int32 indices on the device).
 * Errors: EINVAL (m, n <= 0, nnz < 0, NULL pointers, rowptr not
 * non-decreasing from 0 to nnz, a column index outside [0, n), non-finite
 * values, invalid params), ENOMEM, EDEVICE.  On error *out is set to NULL. */
int pogs_init_sparse(pogs_ctx **out, int64_t m, int64_t n, int64_t nnz, const int64_t *rowptr,
                     const int32_t *colind, const void *val, pogs_dtype dt, pogs_mem mem,
                     const pogs_params *params, void *stream);

/* Solve with functions f (len m) and g (len n) on the context's matrix.
 * params may be NULL (the context's).
 * Warm start (Section 5: the caller may supply x0 and nu0): x0 (len n) and
 * nu0 (len m), in the context's dtype and in the memory space out->mem says,
 * are a primal point and a dual estimate in the original variables; either
 * may be NULL.  The state they define: x = E^-1 x0 and y = A^ x on the graph,
 * y~ = -(D^-1 nu0)/rho0 (the scaled dual the prox step returns when it leaves
 * y unchanged) and x~ = -A^T y~ (the relation every projection restores);
 * from an optimal pair this state is a fixed point and the solve stops after
 * one iteration.  When only one is given the other is estimated (Section 5),
 * as one proximal point step from zero: x0 only -> y~ = prox_f^(y) - y
 * (rho0), then x~ = -A^T y~; nu0 only -> x = prox_g^(-x~), then y = A^ x.
 * Both NULL is the cold start of Algorithm 1.
 * The projection is params->projection: a context set up for the direct
 * projection also runs CGLS solves; a context set up for CGLS only runs CGLS.
 * params->stop_rule selects the residual or the gap test (see pogs_stop_rule).
 * Errors: EINVAL (NULL ctx/f/g/out, wrong lengths, c < 0, e < 0, a == 0 with
 * c > 0, unknown h, non-finite parameters), EUNSUPPORTED (direct projection
 * on a context set up for CGLS, the gap rule with CGLS), EDEVICE. */
int pogs_solve(pogs_ctx *ctx, const pogs_fn *f, const pogs_fn *g, const pogs_params *params,
               const void *x0, const void *nu0, pogs_result *out);

/* Solve R problems that share the context's matrix (a lambda path): problem r
 * uses f[r], g[r] and writes out[r].  The R right-hand sides are stacked so the
 * two passes over A are matrix-matrix products (one read of A per pass for
 * all R problems); each problem keeps its own rho, stopping test and status,
 * exactly as if solved alone up to rounding.  1 <= R <= 256.  Direct
 * projection and the residual test only.
 * Errors as pogs_solve; EUNSUPPORTED for m < n, params->projection ==
 * POGS_PROJ_CGLS, params->stop_rule == POGS_STOP_GAP or a context set up for
 * CGLS. */
int pogs_solve_path(pogs_ctx *ctx, int32_t R, const pogs_fn *f, const pogs_fn *g,
                    const pogs_params *params, pogs_result *out);

/* Release a context and all its device memory.  NULL is a no-op. */
int pogs_free(pogs_ctx *ctx);

/* ---- primitives on a context (each one step of the method) -------------- */

/* Copy the diagonal pre-conditioners D (m entries) and E (n entries) of
 * Section 4.1 (after the Frobenius normalisation) into D, E (float64, memory
 * `mem`).  Either pointer may be NULL. */
int pogs_get_scaling(pogs_ctx *ctx, double *D, double *E, pogs_mem mem);

/* Orthogonal projection of (c, d) onto the graph {(x, y) : y = A^ x} of the
 * scaled matrix A^ = D A E (Section 3.1 projection, computed by the reduced
 * update of Section 3.5 with the cached factor).  c, x have n entries, d, y
 * have m entries, all of the context's dtype in memory `mem`.
 * EUNSUPPORTED on a context set up for CGLS. */
int pogs_project(pogs_ctx *ctx, const void *c, const void *d, void *x, void *y, pogs_mem mem);

/* Evaluate prox_{f,rho}(v) elementwise (Section 5 formula) on the device for a
 * function of length fn->len: out_i = argmin_y f_i(y) + (rho/2)(y - v_i)^2.
 * v and out have fn->len entries of dtype dt in memory `mem`. */
int pogs_prox(const pogs_fn *fn, pogs_dtype dt, double rho, const void *v, void *out,
              pogs_mem mem, void *stream);

/* pogs_prox for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops or harnesses that forbid hipMalloc): the same
 * values as pogs_prox (bit for bit) with v and out in device memory, and the
 * function's parameters (fn, host memory) copied into a device buffer the
 * library owns instead of new allocations.  That buffer holds
 * POGS_NOALLOC_SCRATCH_BYTES on every GPU the library runs on, from the first
 * call on that GPU until the process ends.  It needs
 *   round256(cnt) + 5 * round256(8 cnt)  bytes,  cnt = fn->len (stride 1) or 1,
 * (a NULL parameter takes none), so per-element functions of up to about
 * 1.6 million entries fit; larger ones return POGS_ETOOBIG and launch nothing.
 * Every call on one GPU shares the buffer: calls that overlap on one GPU (other
 * streams, other host threads) race and must be serialised by the caller.
 * The call returns after its work on `stream` (NULL: the null stream) has
 * finished.  Errors: EINVAL (as pogs_prox, or v / out NULL), ETOOBIG, EDEVICE. */
#define POGS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int pogs_prox_noalloc(const pogs_fn *fn, pogs_dtype dt, double rho, const void *v, void *out,
                      void *stream);

/* Time the per-iteration kernels on this context with HIP events on its
 * stream (a measurement aid for benchmarks).  Requires a previous pogs_solve
 * on the context (its functions and iterate are reused).  With the stop test
 * disabled it runs `reps` full iterations as captured launch sequences, then
 * `reps` back-to-back launches of each iteration kernel alone, and writes
 *   ms[0] average ms per full iteration,
 *   direct projection: ms[1] prox step, ms[2] first pass over A, ms[3] solve
 *   with the cached inverse, ms[4] second pass over A; when m >= n the prox
 *   step runs inside the first pass and its finish (ms[1] = 0, ms[2] covers
 *   both launches), and for float32 A with rows of at most 2048 entries
 *   ms[4] is the one-pass kernel that finishes the iteration and forms the
 *   next one's y-side half step and column sums in the same read of A (ms[2]
 *   then covers the stop test and the finish of those column sums);
 *   CGLS (context set up for it, every projection running cg_max_iter
 *   steps): ms[1] prox step, ms[2] the two passes that start a projection,
 *   ms[3] one CG step (two passes), ms[4] = 0
 *   (average ms per launch sequence).
 * The solver state afterwards is meaningless; the next pogs_solve resets it.
 * Errors: EINVAL (NULL, reps < 1, no previous solve), EDEVICE. */
int pogs_profile_iteration(pogs_ctx *ctx, int32_t reps, double *ms);

/* ---- batched and served solves ------------------------------------------ */

/* One problem for the batch engine (all pointers host memory, copied on
 * submit).  params.projection must be POGS_PROJ_DIRECT and params.stop_rule
 * POGS_STOP_RESIDUAL (EUNSUPPORTED otherwise): the grouped path runs on
 * cached factors and the residual test. */
typedef struct {
  int64_t m, n;
  const void *A;
  pogs_dtype dt;        /* POGS_F32 only */
  pogs_order ord;
  int64_t lda;
  pogs_fn f, g;
  pogs_params params;
} pogs_problem;

typedef struct {
  size_t hbm_budget_bytes;  /* device memory the engine may hold for resident
                               problems; 0 = 80% of free memory at creation */
  int32_t max_slots;        /* problems resident at once, 0 = 1024 */
  int32_t chunk_iters;      /* iterations per scheduling round, 0 = 20 */
  void *stream;             /* NULL = engine's own stream */
} pogs_batch_cfg;

typedef struct pogs_batch pogs_batch;

/* Create a serving engine with its own scheduler thread (continuous
 * batching): queued requests are admitted while the memory budget and the
 * slot count allow, set up together, and advanced in chunks of chunk_iters
 * iterations as one group; finished ones leave after each chunk and queued
 * ones join.  Requests too large for the group (see pogs_solve_batch) or with
 * m n > 16 Mi or min(m, n) > 2048 run on the whole-GPU path on two more
 * threads, each with its own stream.  Admission counts every resident request
 * against hbm_budget_bytes, grouped and whole-GPU alike (a whole-GPU request
 * is charged its matrix, the float64 Gram/factor workspace, K^-1 and its
 * vectors while it runs); the head of the whole-GPU queue waits for memory,
 * and the grouped admission then leaves that memory free for it.  A request
 * whose device setup fails finishes with status POGS_FAILED (code in
 * pogs_result.error).  cfg may be NULL.  POGS_EAGAIN if the engine's own
 * arrays do not fit the budget. */
int pogs_batch_create(pogs_batch **out, const pogs_batch_cfg *cfg);

/* Queue a problem; copies its data.  Returns a ticket in *ticket.
 * POGS_EAGAIN if the problem alone exceeds the memory budget; EINVAL as
 * pogs_init/pogs_solve. */
int pogs_batch_submit(pogs_batch *b, const pogs_problem *p, uint64_t *ticket);

/* Non-blocking: 0 and *out filled (x, y, mu, nu copied into out's buffers,
 * which must be host memory here) when the ticket has finished, 1 while it is
 * pending, POGS_ENOTFOUND for an unknown or already-collected ticket.  A
 * finished ticket is released by the poll that returns 0. */
int pogs_batch_poll(pogs_batch *b, uint64_t ticket, pogs_result *out);

/* Block until every submitted ticket has finished. */
int pogs_batch_wait_all(pogs_batch *b);

/* Cancel a queued or running ticket; its poll then returns status
 * POGS_CANCELLED.  POGS_ENOTFOUND for unknown tickets. */
int pogs_batch_cancel(pogs_batch *b, uint64_t ticket);

/* Stop the scheduler thread and free everything (pending tickets are dropped). */
int pogs_batch_destroy(pogs_batch *b);

/* Solve nprob independent problems (host data) in one call.  Problems with
 * n <= 4096 and min(m, n) <= 4096 run as one group: each launch runs one
 * phase (a setup step, or one step of an ADMM iteration) for every problem of
 * the group through a work list of (problem, tile) items, largest problems
 * first; each problem stops at its own stopping test and leaves the group at
 * the next chunk boundary.  Larger problems run one at a time on the
 * whole-GPU path.  A problem gives the same bits alone and in any group.
 * out[i] receives problem i's result (host or device buffers, out[i].mem).
 * Errors as pogs_init/pogs_solve; POGS_EINVAL also for non-finite entries of
 * a grouped matrix (found on the device during the setup). */
int pogs_solve_batch(int32_t nprob, const pogs_problem *probs, pogs_result *out, void *stream);

const char *pogs_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* POGS_H */
