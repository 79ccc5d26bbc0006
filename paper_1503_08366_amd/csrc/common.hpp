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
