// float64 MFMA helpers (v_mfma_f64_16x16x4f64 on gfx950).
//
// Operand layout (same as the f32 16x16x4 form): lane l supplies
//   A[i = l % 16][k = l / 16] and B[k = l / 16][j = l % 16].
// Result layout (differs from the f32 form): lane l, accumulator element r
// holds D[i = 4 r + l / 16][j = l % 16].
#pragma once

#include "common.hpp"

namespace pogs {

typedef double F64Acc __attribute__((ext_vector_type(4)));

__device__ inline F64Acc f64acc_zero() { return F64Acc{0.0, 0.0, 0.0, 0.0}; }

// One K = 4 step of a 32 x 32 wave tile made of 2 x 2 MFMA blocks.
// sa[k][i] and sb[k][j] are k-major LDS stages.
template <int LS>
__device__ inline void f64_tile_step(F64Acc acc[2][2], const double (*sa)[LS], const double (*sb)[LS], int k4,
                                     int ibase, int jbase) {
  const int lane = threadIdx.x & 63;
  const int kr = k4 + (lane >> 4), cl = lane & 15;
  double a[2], b[2];
#pragma unroll
  for (int x = 0; x < 2; ++x) {
    a[x] = sa[kr][ibase + x * 16 + cl];
    b[x] = sb[kr][jbase + x * 16 + cl];
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
}

template <int LS>
__device__ inline void f64_tile_step(F64Acc acc[2][2], double (*sa)[LS], double (*sb)[LS], int k4, int ibase,
                                     int jbase) {
  f64_tile_step<LS>(acc, (const double(*)[LS])sa, (const double(*)[LS])sb, k4, ibase, jbase);
}

// Visit every element of the wave's 32 x 32 tile: fn(row, col, value).
template <class Fn>
__device__ inline void f64_tile_store(const F64Acc acc[2][2], int ibase, int jbase, Fn fn) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) fn(ibase + i * 16 + 4 * r + (lane >> 4), jbase + j * 16 + (lane & 15), acc[i][j][r]);
}

}  // namespace pogs
