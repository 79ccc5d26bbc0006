// Internal structures shared by the kernels' host launchers and the C ABI.
#pragma once

#include <algorithm>

#include "common.hpp"
#include "../../include/pogs.h"

namespace pogs {

// Solver state between iterations (Algorithm 3 and the stop test).
struct CtrlState {
  double rho;       // penalty for the next prox step
  double rescale;   // factor the next prox step applies to (x~, y~) (Section 3.2)
  double r_pri, r_dual, eps_pri, eps_dual;  // residuals of the last finished iteration
  int k;            // iterations whose stop test has run
  int l, u;         // Algorithm 3 markers
  int done;         // 0 running, else 1 + pogs status
  int pending;      // 1: the partial sums of iteration k wait for their stop test
  int by_gap;       // stopped by the gap test: the result is (x, y, -rho x~, -rho y~)
  int spec;         // one-pass iteration: this iteration's y-side half step and column sums
                    // are the ones the previous iteration computed with an unchanged rho
  double eta, eps_gap;  // gap of the state after k iterations and its tolerance (gap rule)
};

// State of the CGLS projection (Section 3.5, indirect) of the current
// iteration; step j's scalars are stored by step parity where a kernel reads
// the previous step's value while its workgroup 0 stores the new one.
struct CgState {
  double alpha;      // step length of the last CG step (its r1 update is pending)
  double gamma[2];   // ||s_j||^2
  double pnorm2[2];  // ||p_j||^2
  double thr2;       // (cg_tol * eps_dual / rho)^2 of this projection
  int stop;          // step at which this projection's CGLS stopped, -1 while running
  int steps_total;   // CG steps over the solve
  int cap_hits;      // projections that stopped at the step cap
  int pad;
};

// Device control block of one solve.  The state is double-buffered by the
// parity of the iteration: the prox step of iteration i reads st[1 - i % 2]
// (the state after iteration i - 1's kernels), runs iteration i - 1's stop
// test and Algorithm 3 itself (every workgroup computes the same values from
// the same partial sums; workgroup 0 stores them) and writes st[i % 2].  So
// no separate control launch is needed per iteration.
struct Ctrl {
  double eps_abs, eps_rel, alpha, delta, tau;
  int max_iter;
  int adaptive;
  CtrlState st[2];
  double cg_tol;  // CGLS tolerance factor (projection = CGLS)
  int cg_cap;     // CGLS step cap per projection
  int stop_gap;   // 1: gap-based stopping (Section 3.4) instead of the residual test
  CgState cg;
  double spec_rho[2];  // one-pass iteration: the rho with which the previous iteration's
                       // one-pass kernel formed the half step of parity i's iteration
};

// Separable function as device arrays (per element).
template <typename T> struct FnDev {
  const uint8_t *h;
  const T *a, *b, *c, *d, *e;
};

// Sparse matrix in compressed rows on the device: row r holds the entries
// ci[rp[r] .. rp[r + 1]) with values va.  The passes over it give each row lpr
// lanes (a power of two up to 64) and launch `grid` workgroups.
// Compressed rows.  nseg > 1 (the copy of A^T): the entries are split by
// column into nseg segments of seg columns each and stored segment by
// segment; the entries of row r in segment s are [rp[s rows + r],
// rp[s rows + r + 1]), so rp has nseg rows + 1 entries.
template <typename T> struct Csr {
  const int *rp;
  const int *ci;
  T *va;
  int rows, lpr, grid, nseg;
};

// Column segments of the sparse A^T: the piece of the gathered vector one
// segment reads (2 values of T per column) is at most kSegBytes, so it stays
// in one XCD's L2 (4 MB) while the grid works on that segment; a workgroup
// keeps the sums of at most kSegRows rows in LDS across the segments.
constexpr size_t kSegBytes = (size_t)1 << 20;
constexpr int kSegRows = 512;
constexpr int kSegGrid = 2048;

// Workgroups of the one-pass tall iteration (tall_one_pass_body) for an m x n
// matrix with leading dimension ld, or 0 where it does not apply (not float32,
// m < n, rows longer than 2048 entries, sparse, or rows over 1024 entries and
// more than 64 rows per wave, which keeps that variant's float32 column sums
// short).  Each workgroup (8 waves) writes one split partial of the column
// sums (2 ld float64 values): 256 of them, as many as are resident at once at
// two waves per SIMD, and at least 64 rows per workgroup so small problems do
// not pay for partials they cannot use.
constexpr int kOnePassWaves = 8;
inline int one_pass_blocks(int64_t m, int64_t n, int ld, int elem_size, bool sparse) {
  if (elem_size != 4 || sparse || m < n || ld > 2048) return 0;
  const int64_t cap = 256;
  if (ld > 1024 && m > 64 * kOnePassWaves * cap) return 0;
  return (int)std::min<int64_t>(cap, std::max<int64_t>(1, (m + 63) / 64));
}

// Default load policy of the passes over A (when not tuned): a matrix larger
// than this is streamed with non-temporal loads (the MI355X last-level cache
// holds 256 MB; below this size A partly stays cached from one pass to the
// next).
constexpr size_t kStreamMatrixBytes = (size_t)192 << 20;

// Everything one iteration of the single-problem pipeline touches.
template <typename T> struct IterArgs {
  int m, n, ld;          // scaled matrix A^ (row-major, leading dim ld)
  int q, ldk;            // (I + G)^{-1}, q = min(m, n), leading dim ldk
  const T *A;
  const T *Kinv;
  FnDev<T> f, g;         // pre-conditioned f^ (length m), g^ (length n)
  T *x, *y, *xt, *yt;    // projected iterate and scaled duals
  T *xh, *yh, *mu, *nu;  // half-step tuple
  T *cx, *dy;            // projection inputs c = x_r + x~, d = y_r + y~
  T *rhs;                // right-hand side of the reduced system (length q)
  double *part;          // gemv_t split partials
  double *s_mu, *s_yh;   // partial sums of mu_h^2, y_h^2 (2 x n_smu, 2 x n_syh: by parity)
  double *s_pri, *s_dual;// partial sums of the residuals
  int nbx, nby;          // prox blocks over x (n) and y (m)
  int n_smu, n_syh;      // slots of s_mu, s_yh per parity: nbx, nby when a prox launch
                         // writes them; finish tiles and row splits in the fused iteration
  int fused;             // 1: the one-pass tall iteration (m >= n, float32, rows of at most
                         // 2048 entries, direct projection, residual stopping)
  T *nyh, *nnu, *ndy;    // the next iteration's half-step set, y side (one-pass iteration)
  int fp_blocks;         // workgroups of the one-pass kernel
  int n_pri, n_dual;     // number of residual partial slots
  Ctrl *ctrl;
  int par;               // parity of this iteration (selects st[] and the prox slots)
  // CGLS projection only: direction p (n), q = A^ p (m), normal residual s (n);
  // per finish-block partials of ||s||^2 and s^T p_prev (2 x n_dual each, by
  // step parity); per row-block partials of ||q||^2 (n_pri)
  T *pv, *qv, *sv;
  double *s_gam, *s_sig, *s_qq;
  // gap rule only: per prox-block partial sums of f^(y) + g^(x) and of
  // f^*(-rho y~) + g^*(-rho x~) for the state entering the prox step
  double *s_gobj, *s_gconj;
  // sparse contexts only: A^ and A^T in compressed rows, and the two vectors
  // the pass over A^T gathers kept interleaved (2 m entries: (r1, nu_h) for
  // the first pass, (r1, q) for the CG steps), one gather per entry
  Csr<T> sa, sat;
  T *pair;
  int nt_rows, nt_cols;  // 1: the row passes (A v) / column passes (A^T v) over A load non-temporally
};

// ---- launchers (setup.hip) ------------------------------------------------
// Convert a matrix (f32/f64, row/col-major, leading dim lda) already on the
// device into row-major T with leading dim ld and zero padding; counts
// non-finite inputs into *bad.
template <typename T>
void launch_layout(const void *src, pogs_dtype sdt, pogs_order ord, int64_t lda, int m, int n,
                   T *dst, int ld, unsigned *bad, hipStream_t s);

// Algorithm 2 sweeps and Frobenius normalisation: fills D (m) and E (n)
// (float64) and scales A in place to D A E.  ws: workspace (see setup.hip).
template <typename T>
int run_equilibrate(T *A, int m, int n, int ld, int iters, double eps_cmp, double *D, double *E,
                    double *ws, size_t ws_bytes, unsigned *counters, hipStream_t s);
size_t equil_workspace_bytes(int m, int n);

// Gram matrix of A^ (A^T A if m >= n else A A^T) plus I, as float64 q x q
// (leading dim ldq = Q, padded to a multiple of 64 with identity).
template <typename T>
int run_gram(const T *A, int m, int n, int ld, double *K, int Q, float *ws32, double *ws64,
             size_t ws_bytes, hipStream_t s);
size_t gram_workspace_bytes(int m, int n, int elem_size);

// Cholesky of K (Q x Q float64, full symmetric; overwritten) and the explicit
// inverse written as T into Kinv (q x q, leading dim ldk).  ws holds
// factor_workspace_bytes(Q).
template <typename T>
int run_factor_inverse(double *K, int q, int Q, T *Kinv, int ldk, double *ws, unsigned *bad,
                       hipStream_t s);
size_t factor_workspace_bytes(int Q);

// ---- launchers (iter.hip) -------------------------------------------------
template <typename T> void launch_scale_fn(const uint8_t *h, const double *a, const double *b,
                                           const double *c, const double *d, const double *e,
                                           const double *scale, bool divide, int len, uint8_t *oh,
                                           T *oa, T *ob, T *oc, T *od, T *oe, hipStream_t s);
template <typename T> void launch_iteration(const IterArgs<T> &p, int splits, int rows_per_split,
                                            int ncolp, hipStream_t s);
// The same iteration with the gap test between the prox step and pass 1.
template <typename T> void launch_iteration_gap(const IterArgs<T> &p, int splits, int rows_per_split,
                                                int ncolp, hipStream_t s);
// The gap test (Section 3.4) on the sums of the prox step just launched: sets
// the stop flag of this iteration when eta < eps_abs + eps_rel |f + g|.
template <typename T> void launch_gap_check(const IterArgs<T> &p, hipStream_t s);
// Run the stop test of the last iteration of a launch sequence whose last
// iteration had parity `par` (writes st[1 - par]); for the host's check.
template <typename T> void launch_control_preview(const IterArgs<T> &p, int par, hipStream_t s);
template <typename T> void launch_iteration_part(const IterArgs<T> &p, int which, int splits, int rows_per_split,
                                                 int ncolp, hipStream_t s);
template <typename T> void launch_project(const IterArgs<T> &p, int splits, int rows_per_split,
                                          int ncolp, const T *c, const T *d, T *x, T *y, hipStream_t s);
// from_state = 0 returns the half-step tuple; 1 returns the state
// (x, y, -rho x~, -rho y~) the gap test accepted.
template <typename T>
void launch_unscale(const IterArgs<T> &p, const double *D, const double *E, const uint8_t *fh0,
                    const double *fa0, const double *fb0, const double *fc0, const double *fd0,
                    const double *fe0, const uint8_t *gh0, const double *ga0, const double *gb0,
                    const double *gc0, const double *gd0, const double *ge0, T *xo, T *yo, T *muo,
                    T *nuo, double *obj_slots, double *obj_out, unsigned *cnt, int from_state, double rho,
                    hipStream_t s);
template <typename T> void launch_prox_eval(const uint8_t *h, const T *a, const T *b, const T *c,
                                            const T *d, const T *e, double rho, const T *v, T *out,
                                            int len, hipStream_t s);

// Warm start of the iteration state from (x0, nu0) (device, original
// variables; either may be NULL): x, y = A^ x, y~, x~ = -A^T y~.
template <typename T>
void launch_warm_start(const IterArgs<T> &p, int splits, int rps, int ncolp, const double *D, const double *E,
                       double rho0, const T *x0, const T *nu0, hipStream_t s);

// CGLS projection (cgls.hip).  One iteration: prox, the first passes, cap
// CG steps (each skipped once the projection's tolerance is met) and a final
// check that applies the last residual update.
template <typename T> void launch_iteration_cg(const IterArgs<T> &p, int splits, int rps, int ncolp, int cap,
                                               hipStream_t s);
// Parts of it for the profiler: 0 prox, 1 first passes, 2 one CG step.
template <typename T> void launch_iteration_cg_part(const IterArgs<T> &p, int which, int splits, int rps,
                                                    int ncolp, hipStream_t s);
// The prox step in the form the CGLS iteration reads its state.
template <typename T> void launch_prox_cg(const IterArgs<T> &p, hipStream_t s);
// State kept by the CGLS iteration from the direct state (x, y, x~, y~):
// c = x + x~, d = y + y~ (then x~ = c - x, y = d - y~ as the prox step reads them).
template <typename T> void launch_cg_from_state(const IterArgs<T> &p, hipStream_t s);

// Row-dot pass shapes (iter.hip).
enum GemvNVariant : int {
  GEMV_N_ROWS1, GEMV_N_ROWS2, GEMV_N_ROWS4, GEMV_N_ROWS8,  // float32, whole rows per wave (NC)
  GEMV_N_L64R1, GEMV_N_L64R4, GEMV_N_L16R1, GEMV_N_L16R4   // LDS-staged vectors (lanes per row, rows)
};
struct GemvNShape {
  int variant;
  int grid;
};
GemvNShape gemv_n_shape(int m, int n, int ld, int elem_size);

// Sparse contexts (sparse.hip).  Lanes per row and grid of the passes over a
// matrix with `rows` rows and `nnz` entries.
void sparse_shape(int rows, int64_t nnz, int *lpr, int *grid);
// Columns per segment of A^T (m columns, n rows, nnz entries, elem bytes per
// value): a kSegBytes piece of the paired vector, with at least two entries
// per row and segment on average (else fewer, wider segments).
int sparse_segment(int m, int n, int64_t nnz, int elem);
// Lanes per row and grid of the segmented pass over A^T (rows * nseg row
// pieces); the grid keeps every workgroup at <= kSegRows rows.
void sparse_seg_shape(int rows, int nseg, int64_t nnz, int *lpr, int *grid);
// Algorithm 2 and the Frobenius normalisation on the sparse pair (A, A^T),
// then both scaled in place to D A E: fills D (m), E (n).  ws: 2 (m + n) + 1024
// doubles.
template <typename T>
void run_equilibrate_sparse(Csr<T> A, Csr<T> At, int m, int n, int iters, double eps_cmp, double *D, double *E,
                            double *ws, hipStream_t s);
// One iteration with the CGLS projection on the sparse pair (two launches per CG step).
template <typename T> void launch_iteration_cg_sparse(const IterArgs<T> &p, int cap, hipStream_t s);
// Parts for the profiler: 0 prox, 1 first passes, 2 one CG step.
template <typename T> void launch_iteration_cg_sparse_part(const IterArgs<T> &p, int which, hipStream_t s);
// Warm start on the sparse pair: the state the dense warm start sets, with
// y = A^ x and x~ = -A^T y~ as row passes over A^ and A^T.
template <typename T>
void launch_warm_start_sparse(const IterArgs<T> &p, const double *D, const double *E, double rho0, const T *x0,
                              const T *nu0, hipStream_t s);

// Iteration geometry helpers.
int gemv_t_tile(int elem_size);
void gemv_t_geometry(int m, int ncols, int elem_size, int *splits, int *rows_per_split, int *ncolp);
int gemv_n_blocks(int m, int ncols, int elem_size, int nrhs_rows_hint);
// Workgroups of `kernel` resident on the whole device at once.
int resident_workgroups(const void *kernel, int block);

}  // namespace pogs
