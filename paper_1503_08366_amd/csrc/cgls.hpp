// Device side of the CGLS projection (Section 3.5, indirect): the epilogues
// and the prologues that decide, from partial sums, whether a CG step runs.
// Shared by the dense launches (cgls.hip) and the sparse ones (sparse.hip).
#pragma once

#include "iter.hpp"

namespace pogs {


// Sum of `len` partials in a fixed order, returned to every thread of the block.
__device__ inline double block_total(const double *slots, int len, double *scratch) {
  double t = 0.0;
  for (int i = threadIdx.x; i < len; i += blockDim.x) t += slots[i];
  t = block_sum(t, scratch);
  __syncthreads();
  if (threadIdx.x == 0) scratch[0] = t;
  __syncthreads();
  return scratch[0];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void prox_cg_kernel(IterArgs<T> p) {
  prox_body<T, true>(hw_block(), p);
}

// C0: t = A^ x_h -> r1 = d - t (kept in yt), (t - y_h)^2 per row
template <typename T> struct EpiCgStart : EpiBase<T> {
  __device__ Pre2<T> pre(int i) const { return Pre2<T>{this->p.dy[i], this->p.yh[i]}; }
  __device__ double row(int i, double t, double, const Pre2<T> &q) const {
    this->p.yt[i] = (T)((double)q.a - t);
    const double r = t - (double)q.b;
    return r * r;
  }
  __device__ double row(int i, double t, double z) const { return row(i, t, z, pre(i)); }
  __device__ void block_done(int b, double v) const { this->p.s_pri[b] = v; }
};

// C1 finish: s_0 = A^T r1 + c - x (x = x_h), (A^T nu_h + mu_h)^2 and s_0^2 per column
template <typename T> struct EpiCgFirst {
  IterArgs<T> p;
  __device__ bool skip() const { return false; }
  __device__ Sum2 column(int j, double w, double z) const {
    const T sv = (T)(w + (double)p.cx[j] - (double)p.x[j]);
    p.sv[j] = sv;
    const double r = z + (double)p.mu[j];
    return Sum2{r * r, (double)sv * (double)sv};
  }
  __device__ void tile_done(int b, double dual, double gam) const {
    p.s_dual[b] = dual;
    p.s_gam[b] = gam;  // step parity 0
  }
};

// Start of the first column pass's finish (every thread): false once the
// solver has stopped; workgroup 0 stores this projection's tolerance
// thr^2 = (cg_tol eps_dual / rho)^2 from this iteration's ||mu_h|| and rho
// and marks the CGLS running.
template <typename T> __device__ bool cg_first_enter(const IterArgs<T> &p) {
  __shared__ double sc[kBlock / kWave];
  if (p.ctrl->st[p.par].done) return false;
  if (blockIdx.x == 0) {
    const double mu2 = block_total(p.s_mu + (size_t)p.par * p.n_smu, p.n_smu, sc);
    if (threadIdx.x == 0) {
      Ctrl &q = *p.ctrl;
      const double eps_dual = q.eps_abs + q.eps_rel * sqrt(mu2);
      const double thr = q.cg_tol * eps_dual / q.st[p.par].rho;
      q.cg.thr2 = thr * thr;
      q.cg.stop = -1;
    }
  }
  return true;
}

// KA epilogue: q_j = A^ s_j + beta q_{j-1}; r1 -= alpha_{j-1} q_{j-1}
template <typename T> struct EpiCgRows {
  IterArgs<T> p;
  double alpha_prev, beta;
  int has_prev;
  __device__ bool skip() const { return false; }
  __device__ Pre2<T> pre(int i) const { return has_prev ? Pre2<T>{p.qv[i], p.yt[i]} : Pre2<T>{T(0), T(0)}; }
  __device__ double row(int i, double as, double, const Pre2<T> &q) const {
    double qn = as;
    if (has_prev) {
      const double qo = (double)q.a;
      p.yt[i] = (T)((double)q.b - alpha_prev * qo);
      qn = as + beta * qo;
    }
    const T qt = (T)qn;
    p.qv[i] = qt;
    return (double)qt * (double)qt;
  }
  __device__ double row(int i, double as, double z) const { return row(i, as, z, pre(i)); }
  __device__ void block_done(int b, double v) const { p.s_qq[b] = v; }
};

// Start of KA (every thread): false when step j does not run.  The step runs
// while j < cap and ||s_j||^2 > thr^2; the first KA that finds it does not
// applies the pending r1 update of step j - 1 (grid-stride over the rows) and
// records where this projection stopped.
template <typename T>
__device__ bool cg_rows_enter(const IterArgs<T> &p, int j, int cap, EpiCgRows<T> *e) {
  __shared__ double sc[kBlock / kWave];
  Ctrl &q = *p.ctrl;
  if (q.st[p.par].done) return false;
  const int stop = q.cg.stop;
  if (stop >= 0 && stop < j) return false;  // stopped at an earlier step
  const double gam = block_total(p.s_gam + (size_t)(j & 1) * p.n_dual, p.n_dual, sc);
  const double alpha_prev = j > 0 ? q.cg.alpha : 0.0;
  const double thr2 = q.cg.thr2;
  if (!(j < cap && gam > thr2)) {
    if (j > 0)
      for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < p.m; i += gridDim.x * blockDim.x)
        p.yt[i] = (T)((double)p.yt[i] - alpha_prev * (double)p.qv[i]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      q.cg.stop = j;
      q.cg.steps_total += j;
      if (gam > thr2) q.cg.cap_hits += 1;
    }
    return false;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) q.cg.gamma[j & 1] = gam;
  e->p = p;
  e->alpha_prev = alpha_prev;
  e->beta = j > 0 ? gam / q.cg.gamma[(j - 1) & 1] : 0.0;
  e->has_prev = j > 0;
  return true;
}

// KB: skipped once the solver or this projection's CGLS has stopped
template <typename T> struct EpiCgSkip {
  IterArgs<T> p;
  __device__ bool skip() const { return p.ctrl->st[p.par].done != 0 || p.ctrl->cg.stop >= 0; }
};

// KC epilogue: p_j, x, s_{j+1}; sums of s_{j+1}^2 and s_{j+1}^T p_j
template <typename T> struct EpiCgStep {
  IterArgs<T> p;
  double alpha, beta;
  int has_prev, next;  // next: step parity of j + 1
  __device__ bool skip() const { return false; }
  __device__ Sum2 column(int i, double w, double z) const {
    double pj = (double)p.sv[i];
    if (has_prev) pj += beta * (double)p.pv[i];
    const T pt = (T)pj;
    p.pv[i] = pt;
    const T xn = (T)((double)p.x[i] + alpha * (double)pt);
    p.x[i] = xn;
    const T sn = (T)(w - alpha * z + (double)p.cx[i] - (double)xn);
    p.sv[i] = sn;
    return Sum2{(double)sn * (double)sn, (double)sn * (double)pt};
  }
  __device__ void tile_done(int b, double gam, double sig) const {
    p.s_gam[(size_t)next * p.n_dual + b] = gam;
    p.s_sig[(size_t)next * p.n_dual + b] = sig;
  }
};


// Start of step j's column finish (every thread): false once the solver or
// this projection's CGLS has stopped; otherwise the epilogue of the step with
// alpha_j = ||s_j||^2 / (||q_j||^2 + ||p_j||^2) and
// ||p_j||^2 = ||s_j||^2 + 2 beta s_j^T p_{j-1} + beta^2 ||p_{j-1}||^2;
// workgroup 0 stores alpha_j and ||p_j||^2.
template <typename T> __device__ bool cg_step_enter(const IterArgs<T> &p, int j, EpiCgStep<T> *e) {
  __shared__ double sc[kBlock / kWave];
  Ctrl &q = *p.ctrl;
  if (q.st[p.par].done || q.cg.stop >= 0) return false;
  const double qq = block_total(p.s_qq, p.n_pri, sc);
  const double gam = q.cg.gamma[j & 1];
  double beta = 0.0, pn2 = gam;
  if (j > 0) {
    beta = gam / q.cg.gamma[(j - 1) & 1];
    const double sig = block_total(p.s_sig + (size_t)(j & 1) * p.n_dual, p.n_dual, sc);
    pn2 = gam + 2.0 * beta * sig + beta * beta * q.cg.pnorm2[(j - 1) & 1];
  }
  const double alpha = gam / (qq + pn2);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    q.cg.alpha = alpha;
    q.cg.pnorm2[j & 1] = pn2;
  }
  *e = EpiCgStep<T>{p, alpha, beta, j > 0 ? 1 : 0, (j + 1) & 1};
  return true;
}

// State kept by the CGLS iteration from the direct state (warm start).
template <typename T>
__global__ __launch_bounds__(kBlock) void cg_from_state_kernel(IterArgs<T> p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p.n) p.cx[i] = p.x[i] + p.xt[i];
  else if (i - p.n < p.m) p.dy[i - p.n] = p.y[i - p.n] + p.yt[i - p.n];
}

}  // namespace pogs
