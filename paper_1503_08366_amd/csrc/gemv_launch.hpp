// Host-side launchers of the matrix-vector passes over the scaled matrix:
// the column-sum pass (split partials, then the finish kernel) and the
// row-dot pass in the variant gemv_n_shape picks.
#pragma once

#include "gemv.hpp"
#include "internal.hpp"

namespace pogs {

// nt: stream the matrix with non-temporal loads (a matrix larger than the
// last-level cache).
template <typename T, typename TV, int NRHS, class Epi>
inline void gemv_t(const T *A, int m, int n, int ld, const TV *v0, const TV *v1, int splits, int rps,
                   double *part, int ncolp, const Epi &epi, hipStream_t s, bool nt = false) {
  const int tile = gemv_t_tile(sizeof(T));
  const int tiles = (int)cdiv(n, tile);
  dim3 grid(tiles, splits);
  if (nt)
    hipLaunchKernelGGL((gemv_t_kernel<T, TV, NRHS, false, Epi, true>), grid, dim3(kBlock), 0, s, A, m, n, ld, v0, v1,
                       rps, part, ncolp, epi);
  else
    hipLaunchKernelGGL((gemv_t_kernel<T, TV, NRHS, false, Epi, false>), grid, dim3(kBlock), 0, s, A, m, n, ld, v0,
                       v1, rps, part, ncolp, epi);
  hipLaunchKernelGGL((gemv_t_finish_kernel<NRHS, Epi>), dim3(cdiv(n, kFinishCols)), dim3(kBlock), 0, s, n, splits,
                     (const double *)part, ncolp, epi);
}

template <typename T, typename TV, int NRHS, class Epi, bool NT>
inline void gemv_n_nt(const T *A, int m, int n, int ld, const TV *v0, const TV *v1, const Epi &epi, hipStream_t s) {
  static_assert(sizeof(T) == sizeof(TV), "matrix and vectors share the element type");
  const GemvNShape sh = gemv_n_shape(m, n, ld, sizeof(T));
  const dim3 grid(sh.grid), block(kBlock);
  if constexpr (sizeof(T) == 4) {
    const float *Af = (const float *)A, *x0 = (const float *)v0, *x1 = (const float *)v1;
    switch (sh.variant) {
      case GEMV_N_ROWS1: hipLaunchKernelGGL((gemv_n_rows_kernel<NRHS, 1, Epi, NT>), grid, block, 0, s, Af, m, n, ld, x0, x1, epi); return;
      case GEMV_N_ROWS2: hipLaunchKernelGGL((gemv_n_rows_kernel<NRHS, 2, Epi, NT>), grid, block, 0, s, Af, m, n, ld, x0, x1, epi); return;
      case GEMV_N_ROWS4: hipLaunchKernelGGL((gemv_n_rows_kernel<NRHS, 4, Epi, NT>), grid, block, 0, s, Af, m, n, ld, x0, x1, epi); return;
      case GEMV_N_ROWS8: hipLaunchKernelGGL((gemv_n_rows_kernel<NRHS, 8, Epi, NT>), grid, block, 0, s, Af, m, n, ld, x0, x1, epi); return;
      default: break;
    }
  }
  switch (sh.variant) {
    case GEMV_N_L64R4:
      hipLaunchKernelGGL((gemv_n_kernel<T, TV, NRHS, false, 64, 4, Epi, NT>), grid, block, 0, s, A, m, n, ld, v0, v1, epi);
      break;
    case GEMV_N_L64R1:
      hipLaunchKernelGGL((gemv_n_kernel<T, TV, NRHS, false, 64, 1, Epi, NT>), grid, block, 0, s, A, m, n, ld, v0, v1, epi);
      break;
    case GEMV_N_L16R4:
      hipLaunchKernelGGL((gemv_n_kernel<T, TV, NRHS, false, 16, 4, Epi, NT>), grid, block, 0, s, A, m, n, ld, v0, v1, epi);
      break;
    default:
      hipLaunchKernelGGL((gemv_n_kernel<T, TV, NRHS, false, 16, 1, Epi, NT>), grid, block, 0, s, A, m, n, ld, v0, v1, epi);
      break;
  }
}

template <typename T, typename TV, int NRHS, class Epi>
inline void gemv_n(const T *A, int m, int n, int ld, const TV *v0, const TV *v1, const Epi &epi, hipStream_t s,
                   bool nt = false) {
  if (nt) gemv_n_nt<T, TV, NRHS, Epi, true>(A, m, n, ld, v0, v1, epi, s);
  else gemv_n_nt<T, TV, NRHS, Epi, false>(A, m, n, ld, v0, v1, epi, s);
}

}  // namespace pogs
