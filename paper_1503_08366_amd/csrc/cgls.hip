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
#include "cgls.hpp"
#include "gemv_launch.hpp"

namespace pogs {

template <typename T>
__global__ __launch_bounds__(kBlock) void cg_first_finish_kernel(IterArgs<T> p, int splits, int ncolp) {
  if (!cg_first_enter<T>(p)) return;
  EpiCgFirst<T> e{p};
  gemv_t_finish_body<2, EpiCgFirst<T>>(hw_block(), p.n, splits, p.part, ncolp, e);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void cg_finish_kernel(IterArgs<T> p, int j, int splits, int ncolp) {
  EpiCgStep<T> e;
  if (!cg_step_enter<T>(p, j, &e)) return;
  gemv_t_finish_body<2, EpiCgStep<T>>(hw_block(), p.n, splits, p.part, ncolp, e);
}

template <int NC, bool NT>
__global__ __launch_bounds__(kBlock) void cg_rows_f32_kernel(IterArgs<float> p, int j, int cap) {
  EpiCgRows<float> e;
  if (!cg_rows_enter<float>(p, j, cap, &e)) return;
  gemv_n_rows_body<1, NC, EpiCgRows<float>, NT>(hw_block(), p.A, p.m, p.n, p.ld, p.sv, p.sv, e);
}

template <typename T, int LPR, int RPT, bool NT>
__global__ __launch_bounds__(kBlock) void cg_rows_lds_kernel(IterArgs<T> p, int j, int cap) {
  EpiCgRows<T> e;
  if (!cg_rows_enter<T>(p, j, cap, &e)) return;
  gemv_n_body<T, T, 1, false, LPR, RPT, EpiCgRows<T>, NT>(hw_block(), p.A, p.m, p.n, p.ld, p.sv, p.sv, e);
}

template <typename T, bool NT> static void launch_cg_rows_nt(const IterArgs<T> &p, int j, int cap, hipStream_t s) {
  const GemvNShape sh = gemv_n_shape(p.m, p.n, p.ld, sizeof(T));
  const dim3 grid(sh.grid), block(kBlock);
  if constexpr (sizeof(T) == 4) {
    switch (sh.variant) {
      case GEMV_N_ROWS1: hipLaunchKernelGGL((cg_rows_f32_kernel<1, NT>), grid, block, 0, s, p, j, cap); return;
      case GEMV_N_ROWS2: hipLaunchKernelGGL((cg_rows_f32_kernel<2, NT>), grid, block, 0, s, p, j, cap); return;
      case GEMV_N_ROWS4: hipLaunchKernelGGL((cg_rows_f32_kernel<4, NT>), grid, block, 0, s, p, j, cap); return;
      case GEMV_N_ROWS8: hipLaunchKernelGGL((cg_rows_f32_kernel<8, NT>), grid, block, 0, s, p, j, cap); return;
      default: break;
    }
  }
  switch (sh.variant) {
    case GEMV_N_L64R4: hipLaunchKernelGGL((cg_rows_lds_kernel<T, 64, 4, NT>), grid, block, 0, s, p, j, cap); break;
    case GEMV_N_L64R1: hipLaunchKernelGGL((cg_rows_lds_kernel<T, 64, 1, NT>), grid, block, 0, s, p, j, cap); break;
    case GEMV_N_L16R4: hipLaunchKernelGGL((cg_rows_lds_kernel<T, 16, 4, NT>), grid, block, 0, s, p, j, cap); break;
    default: hipLaunchKernelGGL((cg_rows_lds_kernel<T, 16, 1, NT>), grid, block, 0, s, p, j, cap); break;
  }
}

template <typename T> static void launch_cg_rows(const IterArgs<T> &p, int j, int cap, hipStream_t s) {
  if (p.nt_rows) launch_cg_rows_nt<T, true>(p, j, cap, s);
  else launch_cg_rows_nt<T, false>(p, j, cap, s);
}

template <typename T> static void launch_first(const IterArgs<T> &p, int splits, int rps, int ncolp, hipStream_t s) {
  EpiCgStart<T> e0{{p}};
  gemv_n<T, T, 1>(p.A, p.m, p.n, p.ld, p.x, p.x, e0, s, p.nt_rows);
  const int tiles = (int)cdiv(p.n, gemv_t_tile(sizeof(T)));
  EpiBase<T> eb{p};
  if (p.nt_cols)
    hipLaunchKernelGGL((gemv_t_kernel<T, T, 2, false, EpiBase<T>, true>), dim3(tiles, splits), dim3(kBlock), 0, s, p.A,
                       p.m, p.n, p.ld, (const T *)p.yt, (const T *)p.nu, rps, p.part, ncolp, eb);
  else
    hipLaunchKernelGGL((gemv_t_kernel<T, T, 2, false, EpiBase<T>, false>), dim3(tiles, splits), dim3(kBlock), 0, s,
                       p.A, p.m, p.n, p.ld, (const T *)p.yt, (const T *)p.nu, rps, p.part, ncolp, eb);
  hipLaunchKernelGGL(cg_first_finish_kernel<T>, dim3(cdiv(p.n, kFinishCols)), dim3(kBlock), 0, s, p, splits, ncolp);
}

template <typename T> static void launch_step(const IterArgs<T> &p, int j, int cap, int splits, int rps, int ncolp,
                                              hipStream_t s) {
  launch_cg_rows<T>(p, j, cap, s);
  const int tiles = (int)cdiv(p.n, gemv_t_tile(sizeof(T)));
  EpiCgSkip<T> ek{p};
  if (p.nt_cols)
    hipLaunchKernelGGL((gemv_t_kernel<T, T, 2, false, EpiCgSkip<T>, true>), dim3(tiles, splits), dim3(kBlock), 0, s,
                       p.A, p.m, p.n, p.ld, (const T *)p.yt, (const T *)p.qv, rps, p.part, ncolp, ek);
  else
    hipLaunchKernelGGL((gemv_t_kernel<T, T, 2, false, EpiCgSkip<T>, false>), dim3(tiles, splits), dim3(kBlock), 0, s,
                       p.A, p.m, p.n, p.ld, (const T *)p.yt, (const T *)p.qv, rps, p.part, ncolp, ek);
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

template <typename T> void launch_prox_cg(const IterArgs<T> &p, hipStream_t s) {
  hipLaunchKernelGGL(prox_cg_kernel<T>, dim3(p.nbx + p.nby), dim3(kBlock), 0, s, p);
}

template <typename T> void launch_cg_from_state(const IterArgs<T> &p, hipStream_t s) {
  hipLaunchKernelGGL(cg_from_state_kernel<T>, dim3(cdiv(p.n + p.m, kBlock)), dim3(kBlock), 0, s, p);
}

template void launch_iteration_cg<float>(const IterArgs<float> &, int, int, int, int, hipStream_t);
template void launch_iteration_cg<double>(const IterArgs<double> &, int, int, int, int, hipStream_t);
template void launch_iteration_cg_part<float>(const IterArgs<float> &, int, int, int, int, hipStream_t);
template void launch_iteration_cg_part<double>(const IterArgs<double> &, int, int, int, int, hipStream_t);
template void launch_prox_cg<float>(const IterArgs<float> &, hipStream_t);
template void launch_prox_cg<double>(const IterArgs<double> &, hipStream_t);
template void launch_cg_from_state<float>(const IterArgs<float> &, hipStream_t);
template void launch_cg_from_state<double>(const IterArgs<double> &, hipStream_t);

}  // namespace pogs
