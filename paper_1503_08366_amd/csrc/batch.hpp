// Batched solver: one workgroup solves one problem end to end (setup and ADMM
// iterations), pulling problems from a device work queue.  Shared by the
// one-call batch entry point and the serving engine.
#pragma once

#include "internal.hpp"

namespace pogs {

// Largest sizes the one-workgroup path takes (larger problems use the
// whole-GPU path).
constexpr int kBatchMaxQ = 2048;  // min(m, n)
constexpr int kBatchMaxN = 8192;  // n (vectors staged in LDS)

// One problem of a batch, in device memory.  Sizes and pointers are set by
// the host; the solver fields are written by the device.
struct BProb {
  int m, n, ld, q, ldk, Q;
  float *A;                 // m x ld: raw, scaled to D A E in place by the setup
  float *Kinv;              // q x ldk
  double *D, *E;
  const uint8_t *fh, *gh;   // base-function codes
  const double *f0, *g0;    // original parameters a, b, c, d, e (5 x m, 5 x n)
  float *fs, *gs;           // pre-conditioned parameters (5 x m, 5 x n)
  float *vec;               // x, xt, xh, mu, cx (n each, stride ldn); y, yt, yh, nu, dy (stride ldm); rhs (q)
  float *out;               // returned x (n), y (m), mu (n), nu (m)
  int ldn, ldm;
  // parameters
  double eps_abs, eps_rel, rho0, alpha, delta, tau, gamma;
  int max_iter, adaptive, equil_iters, pad0;
  // solver state (device-written)
  double rho, rescale;
  int k, l, u;
  int status;               // -1 running, else pogs status
  int setup_done;
  unsigned bad;             // non-finite A or failed factorisation
  double r_pri, r_dual, eps_pri, eps_dual, optval;
};

// Launch the persistent batch kernel: problems order[0..count) (device index
// list into probs) are taken from the queue counter *next (zeroed by the
// caller) by `slots` workgroups; each workgroup uses `slot_doubles` doubles of
// `scratch`.  Each problem runs at most iter_budget iterations in this launch.
void launch_batch(BProb *probs, const int *order, int count, unsigned *next, double *scratch, size_t slot_doubles,
                  int slots, int max_n, int iter_budget, hipStream_t s);

size_t batch_slot_doubles(int Qmax);
size_t batch_lds_bytes(int max_n);

}  // namespace pogs
