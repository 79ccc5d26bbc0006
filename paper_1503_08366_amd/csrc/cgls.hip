// Indirect projection (Section 3.5): each ADMM iteration projects onto the
// graph by CGLS on the reduced least-squares problem
//     x = argmin ||x - c||^2 + ||A^ x - d||^2     ([A^; I] x ~ [d; c]),
// started from the half step x_h, with no Gram matrix and no factorisation.
//
// Per iteration (after the prox step, which also sets x = x_h):
//   C0   row pass     t = A^ x_h         -> r1 = d - t, primal residual sums
//   C1   column pass  A^T [r1, nu_h]     -> s = A^T r1 + c - x, dual residual sums
//   then CG steps j = 0, 1, ..., cap - 1, three launches each:
//   KA   row pass     q_j = A^ s_j + beta q_{j-1}  (= A^ p_j), r1 -= alpha_{j-1} q_{j-1},
//                     ||q_j||^2 sums; the step runs only while ||s_j|| > thr
//   KB   column pass  A^T [r1, q_j] split partials
//   KC   finish       p_j = s_j + beta p_{j-1}, x += alpha_j p_j,
//                     s_{j+1} = A^T r1 - alpha_j A^T q_j + c - x
//   and a last KA (j = cap) that only applies the pending r1 update.
// alpha_j = ||s_j||^2 / (||q_j||^2 + ||p_j||^2), beta = ||s_j||^2 / ||s_{j-1}||^2,
// with ||p_j||^2 = ||s_j||^2 + 2 beta s_j^T p_{j-1} + beta^2 ||p_{j-1}||^2 (the
// expansion of ||s_j + beta p_{j-1}||^2, whose terms the previous finish
// summed), so every scalar is known at the start of the launch that needs it.
// The projection leaves x~ = c - x, y~ = r1, y = d - r1 (the prox step reads
// them in that form).  The tolerance is thr = cg_tol * eps_dual / rho: the
// final normal residual s equals x~ + A^T y~, which enters the next dual
// residual multiplied by rho.
//
// Every launch of a step decides from the same partial sums whether the step
// runs, so the sequence of launches is fixed (it can be captured once) while
// the work stops as soon as the tolerance is met.
#include "iter.hpp"
#include "gemv_launch.hpp"

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

template <typename T>
__global__ __launch_bounds__(kBlock) void cg_first_finish_kernel(IterArgs<T> p, int splits, int ncolp) {
  __shared__ double sc[kBlock / kWave];
  if (p.ctrl->st[p.par].done) return;
  if (blockIdx.x == 0) {
    // tolerance of this projection from this iteration's ||mu_h|| and rho
    const double mu2 = block_total(p.s_mu + (size_t)p.par * p.nbx, p.nbx, sc);
    if (threadIdx.x == 0) {
      Ctrl &q = *p.ctrl;
      const double eps_dual = q.eps_abs + q.eps_rel * sqrt(mu2);
      const double thr = q.cg_tol * eps_dual / q.st[p.par].rho;
      q.cg.thr2 = thr * thr;
      q.cg.stop = -1;
    }
  }
  EpiCgFirst<T> e{p};
  gemv_t_finish_body<2, EpiCgFirst<T>>(hw_block(), p.n, splits, p.part, ncolp, e);
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

template <int NC>
__global__ __launch_bounds__(kBlock) void cg_rows_f32_kernel(IterArgs<float> p, int j, int cap) {
  EpiCgRows<float> e;
  if (!cg_rows_enter<float>(p, j, cap, &e)) return;
  gemv_n_rows_body<1, NC, EpiCgRows<float>>(hw_block(), p.A, p.m, p.n, p.ld, p.sv, p.sv, e);
}

template <typename T, int LPR, int RPT>
__global__ __launch_bounds__(kBlock) void cg_rows_lds_kernel(IterArgs<T> p, int j, int cap) {
  EpiCgRows<T> e;
  if (!cg_rows_enter<T>(p, j, cap, &e)) return;
  gemv_n_body<T, T, 1, false, LPR, RPT, EpiCgRows<T>>(hw_block(), p.A, p.m, p.n, p.ld, p.sv, p.sv, e);
}

template <typename T> static void launch_cg_rows(const IterArgs<T> &p, int j, int cap, hipStream_t s) {
  const GemvNShape sh = gemv_n_shape(p.m, p.n, p.ld, sizeof(T));
  const dim3 grid(sh.grid), block(kBlock);
  if constexpr (sizeof(T) == 4) {
    switch (sh.variant) {
      case GEMV_N_ROWS1: hipLaunchKernelGGL(cg_rows_f32_kernel<1>, grid, block, 0, s, p, j, cap); return;
      case GEMV_N_ROWS2: hipLaunchKernelGGL(cg_rows_f32_kernel<2>, grid, block, 0, s, p, j, cap); return;
      case GEMV_N_ROWS4: hipLaunchKernelGGL(cg_rows_f32_kernel<4>, grid, block, 0, s, p, j, cap); return;
      case GEMV_N_ROWS8: hipLaunchKernelGGL(cg_rows_f32_kernel<8>, grid, block, 0, s, p, j, cap); return;
      default: break;
    }
  }
  switch (sh.variant) {
    case GEMV_N_L64R4: hipLaunchKernelGGL((cg_rows_lds_kernel<T, 64, 4>), grid, block, 0, s, p, j, cap); break;
    case GEMV_N_L64R1: hipLaunchKernelGGL((cg_rows_lds_kernel<T, 64, 1>), grid, block, 0, s, p, j, cap); break;
    case GEMV_N_L16R4: hipLaunchKernelGGL((cg_rows_lds_kernel<T, 16, 4>), grid, block, 0, s, p, j, cap); break;
    default: hipLaunchKernelGGL((cg_rows_lds_kernel<T, 16, 1>), grid, block, 0, s, p, j, cap); break;
  }
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

template <typename T>
__global__ __launch_bounds__(kBlock) void cg_finish_kernel(IterArgs<T> p, int j, int splits, int ncolp) {
  __shared__ double sc[kBlock / kWave];
  Ctrl &q = *p.ctrl;
  if (q.st[p.par].done || q.cg.stop >= 0) return;
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
  EpiCgStep<T> e{p, alpha, beta, j > 0 ? 1 : 0, (j + 1) & 1};
  gemv_t_finish_body<2, EpiCgStep<T>>(hw_block(), p.n, splits, p.part, ncolp, e);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void cg_from_state_kernel(IterArgs<T> p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p.n) p.cx[i] = p.x[i] + p.xt[i];
  else if (i - p.n < p.m) p.dy[i - p.n] = p.y[i - p.n] + p.yt[i - p.n];
}

template <typename T> static void launch_first(const IterArgs<T> &p, int splits, int rps, int ncolp, hipStream_t s) {
  EpiCgStart<T> e0{{p}};
  gemv_n<T, T, 1>(p.A, p.m, p.n, p.ld, p.x, p.x, e0, s);
  const int tiles = (int)cdiv(p.n, gemv_t_tile(sizeof(T)));
  EpiBase<T> eb{p};
  hipLaunchKernelGGL((gemv_t_kernel<T, T, 2, false, EpiBase<T>>), dim3(tiles, splits), dim3(kBlock), 0, s, p.A, p.m,
                     p.n, p.ld, (const T *)p.yt, (const T *)p.nu, rps, p.part, ncolp, eb);
  hipLaunchKernelGGL(cg_first_finish_kernel<T>, dim3(cdiv(p.n, kFinishCols)), dim3(kBlock), 0, s, p, splits, ncolp);
}

template <typename T> static void launch_step(const IterArgs<T> &p, int j, int cap, int splits, int rps, int ncolp,
                                              hipStream_t s) {
  launch_cg_rows<T>(p, j, cap, s);
  const int tiles = (int)cdiv(p.n, gemv_t_tile(sizeof(T)));
  EpiCgSkip<T> ek{p};
  hipLaunchKernelGGL((gemv_t_kernel<T, T, 2, false, EpiCgSkip<T>>), dim3(tiles, splits), dim3(kBlock), 0, s, p.A,
                     p.m, p.n, p.ld, (const T *)p.yt, (const T *)p.qv, rps, p.part, ncolp, ek);
  hipLaunchKernelGGL(cg_finish_kernel<T>, dim3(cdiv(p.n, kFinishCols)), dim3(kBlock), 0, s, p, j, splits, ncolp);
}

template <typename T>
void launch_iteration_cg(const IterArgs<T> &p, int splits, int rps, int ncolp, int cap, hipStream_t s) {
  hipLaunchKernelGGL(prox_cg_kernel<T>, dim3(p.nbx + p.nby), dim3(kBlock), 0, s, p);
  launch_first<T>(p, splits, rps, ncolp, s);
  for (int j = 0; j < cap; ++j) launch_step<T>(p, j, cap, splits, rps, ncolp, s);
  launch_cg_rows<T>(p, cap, cap, s);
}

template <typename T>
void launch_iteration_cg_part(const IterArgs<T> &p, int which, int splits, int rps, int ncolp, hipStream_t s) {
  if (which == 0) hipLaunchKernelGGL(prox_cg_kernel<T>, dim3(p.nbx + p.nby), dim3(kBlock), 0, s, p);
  else if (which == 1) launch_first<T>(p, splits, rps, ncolp, s);
  else launch_step<T>(p, 0, 1 << 30, splits, rps, ncolp, s);
}

template <typename T> void launch_cg_from_state(const IterArgs<T> &p, hipStream_t s) {
  hipLaunchKernelGGL(cg_from_state_kernel<T>, dim3(cdiv(p.n + p.m, kBlock)), dim3(kBlock), 0, s, p);
}

template void launch_iteration_cg<float>(const IterArgs<float> &, int, int, int, int, hipStream_t);
template void launch_iteration_cg<double>(const IterArgs<double> &, int, int, int, int, hipStream_t);
template void launch_iteration_cg_part<float>(const IterArgs<float> &, int, int, int, int, hipStream_t);
template void launch_iteration_cg_part<double>(const IterArgs<double> &, int, int, int, int, hipStream_t);
template void launch_cg_from_state<float>(const IterArgs<float> &, hipStream_t);
template void launch_cg_from_state<double>(const IterArgs<double> &, hipStream_t);

}  // namespace pogs
