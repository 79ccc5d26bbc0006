// Grouped launches: one launch runs one phase (a setup step or one step of
// an ADMM iteration) for many problems at once.  Each workgroup reads a work
// item (problem, block coordinates) and runs the same device body the
// single-problem launch runs for that block, on that problem's buffers.  So
// every pass over a matrix runs with the whole GPU behind it however small
// the problem is, and the per-launch cost is shared by all problems in the
// group.  A problem's arithmetic does not depend on which other problems
// share its launches (its work items and their order of reduction are a
// function of its own shape), so it gives the same bits alone and in any mix.
#pragma once

#include "internal.hpp"

namespace pogs {

// What the host reads back about each problem after a chunk.
struct GStatus {
  CtrlState st;        // state after the last iteration of the chunk
  unsigned flags[2];   // non-finite entries of A, failed pivots
  double obj;          // objective (valid after G_UNSCALE)
};

// One problem of a group, in device memory (float32 iterations, float64
// factorisation and norms).
struct GProb {
  IterArgs<float> it;        // iteration buffers and sizes (par set per launch)
  int tall;                  // m >= n: K = I + A^T A, else I + A A^T
  int lpr16;                 // rows of A shorter than 512: 16 lanes per row, else 64
  int lpr16k;                // the same for the rows of K^{-1}
  int splits, rps, ncolp;    // column-sum (A^T v) geometry over the n columns
  int Q, nbt;                // factor: Q = round_up(q, 64), nbt = Q / 64 blocks
  int eq_U, eq_rps, eq_nsplit, eq_ncolp;  // Sinkhorn-Knopp sweep geometry
  int equil_iters;
  int lay_rows;              // rows per layout work item (row-major input)
  int colmajor;              // input order
  long long lda;             // input leading dimension
  const float *raw;          // input as uploaded (m x n float32)
  double *D, *E;             // final scaling (Section 4.1)
  double *d, *e, *eq_part, *eq_slots;
  double gamma_m, gamma_n, mf, nf;
  double *K, *X, *Dinv;      // Q x Q, Q x Q, nbt x 64 x 64 (float64 factor workspace)
  unsigned *flags;           // [0] non-finite entries of A, [1] failed pivots
  const uint8_t *fh0, *gh0;  // original functions: codes and a, b, c, d, e (SoA)
  const double *f0, *g0;
  float *out;                // returned x (n) | y (m) | mu (n) | nu (m)
  double *obj, *obj_slots;   // objective and its per-block partial sums
  unsigned *obj_cnt;         // arrival counter of the objective sum
  GStatus *status;           // this problem's entry of the host-visible status array
  // solver parameters (Algorithm 1, Section 3.2, Algorithm 3)
  double eps_abs, eps_rel, alpha, delta, tau, rho0;
  int max_iter, adaptive;
};

// A work item: the problem and the block coordinates of one workgroup.
struct GItem {
  int prob, x, y, nx, ny;
};

enum GPhase : int {
  G_LAYOUT_ROWS = 0,  // row-major input -> padded A, non-finite count, e = 1
  G_LAYOUT_TILES,     // column-major input (32 x 32 tiles)
  G_EQ_SWEEP,         // one Sinkhorn-Knopp sweep (arg: U = ceil(n / 1024), all items of one U)
  G_EQ_COLFINISH,     // column sums -> e, Frobenius partial sums
  G_EQ_NORMALIZE,     // D, E from d, e and the Frobenius norm
  G_SCALE_MATRIX,     // A <- D A E
  G_SCALE_FN,         // pre-conditioned function parameters (y = 0: f, y = 1: g)
  G_GRAM,             // K = I + G, lower triangle, 128 x 128 tiles
  G_TRTRI_INIT,       // X <- I on the lower block triangle
  G_POTRF0,           // factor diagonal block 0
  G_PANEL,            // Cholesky / inverse step, first half (arg: kb)
  G_UPDATE,           // Cholesky / inverse step, second half (arg: kb)
  G_KINV,             // K^{-1} = L^{-T} L^{-1} in float32
  G_PROX,             // prox step (+ stop test of the previous iteration); arg: parity for all below
  G_PASS1_T,          // tall: A^T [d, nu_h] split partials
  G_PASS1_W64,        // wide: A [c, x_h], 64 lanes per row
  G_PASS1_W16,        // wide: A [c, x_h], 16 lanes per row
  G_FINISH1,          // tall: column finish of pass 1
  G_SOLVE64,          // K^{-1} rhs, 64 lanes per row
  G_SOLVE16,          // K^{-1} rhs, 16 lanes per row
  G_PASS2_T64,        // tall: A [x, x_h], 64 lanes per row
  G_PASS2_T16,        // tall: A [x, x_h], 16 lanes per row
  G_PASS2_W,          // wide: A^T [y~, nu_h] split partials
  G_FINISH2,          // wide: column finish of pass 2
  G_PREVIEW,          // stop test of the last iteration of a chunk
  G_UNSCALE,          // original variables and objective
  G_INIT_STATE,       // control block for the first iteration
  G_GATHER,           // state, flags and objective into the status array
  G_NUM_PHASES
};

// Rows per workgroup of the row-dot passes in each variant.
constexpr int kGRows64 = 16;  // 64 lanes per row, 4 rows per wave
constexpr int kGRows16 = 64;  // 16 lanes per row, 4 rows per lane group

void launch_group(int phase, const GProb *probs, const GItem *items, int count, int arg, hipStream_t s);

}  // namespace pogs
