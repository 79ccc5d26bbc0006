// Shared device/host helpers for the gfx950 graph-form ADMM library.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <type_traits>

namespace pogs {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // threads per workgroup of the streaming kernels
constexpr int kFinishCols = 16;  // columns per workgroup when split column sums are finished

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return cdiv(a, b) * b; }

// Element type of 16-byte vector loads: 4 floats or 2 doubles.
template <typename T> struct Vec16;
template <> struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int N = 4;
};
template <> struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int N = 2;
};

// Coordinates of a workgroup's share of a launch: the hardware block index
// for a launch over one problem, or the fields of a work item when one
// launch covers the tiles of many problems.
struct Blk {
  int x, y;    // block index
  int nx, ny;  // blocks of this problem along x and y
};
__device__ inline Blk hw_block() { return Blk{(int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, (int)gridDim.y}; }

// Two sums carried together through a reduction.
struct Sum2 {
  double a, b;
};

// Sum over the 64 lanes of a wave (every lane receives the total).
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum over the 64 lanes of a wave without LDS traffic: DPP exchanges within
// rows of 16 lanes (lanes 1 apart, 2 apart, then the mirror images within 8
// and within 16), then the gfx950 permlane swaps between the two rows of each
// 32-lane half and between the two halves.  Each step adds the two values of
// a lane pair in the same order in both lanes, so every lane ends with the
// same bits.  The order of the additions differs from wave_sum's.  Every
// pattern reads a valid lane, so the DPP moves need no old value.
__device__ inline double dpp_pair_sum(double v, int ctrl) {
  const long long b = __double_as_longlong(v);
  int lo = (int)b, hi = (int)(b >> 32);
  switch (ctrl) {  // the control must be a constant per call site
    case 0xB1: lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xf, 0xf, false);
               hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xf, 0xf, false); break;  // quad_perm 1,0,3,2
    case 0x4E: lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xf, 0xf, false);
               hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xf, 0xf, false); break;  // quad_perm 2,3,0,1
    case 0x141: lo = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xf, 0xf, false);
                hi = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xf, 0xf, false); break;  // row_half_mirror
    default: lo = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xf, 0xf, false);
             hi = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xf, 0xf, false); break;  // row_mirror
  }
  return v + __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
__device__ inline double swap_pair_sum16(double v) {
  const long long b = __double_as_longlong(v);
  const auto l = __builtin_amdgcn_permlane16_swap((unsigned)b, (unsigned)b, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  return __longlong_as_double((long long)l[0] | ((long long)h[0] << 32)) +
         __longlong_as_double((long long)l[1] | ((long long)h[1] << 32));
}
__device__ inline double swap_pair_sum32(double v) {
  const long long b = __double_as_longlong(v);
  const auto l = __builtin_amdgcn_permlane32_swap((unsigned)b, (unsigned)b, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap((unsigned)(b >> 32), (unsigned)(b >> 32), false, false);
  return __longlong_as_double((long long)l[0] | ((long long)h[0] << 32)) +
         __longlong_as_double((long long)l[1] | ((long long)h[1] << 32));
}
__device__ inline double wave_sum_dpp(double v) {
  v = dpp_pair_sum(v, 0xB1);
  v = dpp_pair_sum(v, 0x4E);
  v = dpp_pair_sum(v, 0x141);
  v = dpp_pair_sum(v, 0x140);
  v = swap_pair_sum16(v);
  return swap_pair_sum32(v);
}

// Sum over groups of W consecutive lanes (W a power of two <= 64).
template <int W> __device__ inline double group_sum(double v) {
#pragma unroll
  for (int o = W / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Block-wide sum of one double per thread; the result is valid in thread 0.
// `scratch` holds blockDim.x / 64 doubles of LDS.  Reduction order is fixed
// (wave shuffle tree, then waves in index order), so results are
// deterministic.
__device__ inline double block_sum(double v, double *scratch) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) scratch[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < nw; ++i) t += scratch[i];
  return t;
}

// Loads of data written by other workgroups of the same launch: read at
// device (agent) scope so no stale cache line is returned.
__device__ inline double load_agent(const double *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// "Last workgroup done" protocol: every thread fences its own global writes,
// thread 0 bumps `counter`; returns true (in every thread) for the workgroup
// that arrives last, after an acquire fence.  That workgroup also resets the
// counter for the next launch.  `flag` is one int of LDS.
__device__ inline bool arrive_last(unsigned *counter, unsigned total, int *flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned old = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    *flag = (old == total - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = *flag != 0;
  if (last) {
    __threadfence();
    if (threadIdx.x == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  return last;
}

}  // namespace pogs

#define POGS_HIP_TRY(expr)                                                   \
  do {                                                                       \
    hipError_t _e = (expr);                                                  \
    if (_e != hipSuccess) {                                                  \
      fprintf(stderr, "pogs: %s failed: %s (%s:%d)\n", #expr,                \
              hipGetErrorString(_e), __FILE__, __LINE__);                    \
      return POGS_EDEVICE;                                                   \
    }                                                                        \
  } while (0)
