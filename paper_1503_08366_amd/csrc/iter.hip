// One ADMM iteration of the single-problem pipeline on gfx950 (Algorithm 1 with
// the Section 3.2 over-relaxation, Section 3.3 half-step duals, Section 3.4
// residual stopping and Algorithm 3 adaptive rho), as four steps (five
// launches: the pass that sums columns of A finishes in a second small kernel):
//
//   1. prox      : x_h = prox_g^(x - x~), y_h = prox_f^(y - y~), mu_h, nu_h,
//                  relaxed c = x_r + x~, d = y_r + y~, partial ||mu_h||^2, ||y_h||^2
//   2. pass 1    : m >= n: [w, s] = A^T [d, nu_h] -> rhs = c + w, (s + mu_h)^2
//                  m <  n: [u, t] = A   [c, x_h]  -> rhs = u - d, (t - y_h)^2
//   3. solve     : m >= n: x = K^{-1} rhs, x~ = c - x
//                  m <  n: y = d + K^{-1} rhs, y~ = d - y
//   4. pass 2    : m >= n: [y, t] = A [x, x_h] -> y~ = d - y, (t - y_h)^2
//                  m <  n: [z, s] = A^T [y~, nu_h] -> x = c + z, x~ = c - x, (s + mu_h)^2
// The stop test and Algorithm 3 of iteration i run at the start of iteration
// i + 1's prox step, in every workgroup, from the partial sums in a fixed order
// (see Ctrl); a one-workgroup kernel runs it after the last iteration of a
// launch sequence so the host can see the stop flag.
//
// The reduced update is the one of Section 3.5 with K = I + A^T A (m >= n) or
// I + A A^T (m < n); K^{-1} is formed once from the float64 Cholesky factor.
// The wide-case x update is c + A^T (d - y), the sign the projection's
// optimality conditions give.
#include "iter.hpp"
#include "gemv_launch.hpp"

namespace pogs {

template <typename T>
__global__ __launch_bounds__(kBlock) void control_preview_kernel(IterArgs<T> p, int par) {
  control_preview_body<T>(p, par);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void prox_kernel(IterArgs<T> p) {
  prox_body<T>(hw_block(), p);
}

template <typename T, bool NT>
__global__ __launch_bounds__(kBlock) void tall_pass1_prox_kernel(IterArgs<T> p, int rps, int ncolp) {
  tall_pass1_prox_body<T, NT>(hw_block(), p, rps, ncolp);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void tall_finish_prox_kernel(IterArgs<T> p, int splits, int ncolp) {
  tall_finish_prox_body<T>(hw_block(), p, splits, ncolp);
}

template <int NC, bool NT>
__global__ __launch_bounds__(kOnePassThreads) void tall_one_pass_kernel(IterArgs<float> p, int ncolp) {
  tall_one_pass_body<NC, NT>(hw_block(), p, ncolp);
}

template <bool NT> static void launch_one_pass_nt(const IterArgs<float> &p, int ncolp, hipStream_t s) {
  const dim3 grid((unsigned)p.fp_blocks), block(kOnePassThreads);
  if (p.ld <= 256) hipLaunchKernelGGL((tall_one_pass_kernel<1, NT>), grid, block, 0, s, p, ncolp);
  else if (p.ld <= 512) hipLaunchKernelGGL((tall_one_pass_kernel<2, NT>), grid, block, 0, s, p, ncolp);
  else if (p.ld <= 1024) hipLaunchKernelGGL((tall_one_pass_kernel<4, NT>), grid, block, 0, s, p, ncolp);
  else hipLaunchKernelGGL((tall_one_pass_kernel<8, NT>), grid, block, 0, s, p, ncolp);
}

// Standalone projection (no solver state): outputs go to caller buffers.
template <typename T> struct ProjArgs {
  const T *c, *d;
  T *x, *y;
  T *rhs;
};
template <typename T> struct EpiNoSkip {
  __device__ bool skip() const { return false; }
};
template <typename T> struct EpiProjTall1 : EpiNoSkip<T> {  // rhs = c + A^T d
  ProjArgs<T> a;
  __device__ double column(int j, double w, double) const { a.rhs[j] = (T)((double)a.c[j] + w); return 0.0; }
  __device__ void tile_done(int, double) const {}
};
template <typename T> struct EpiProjTallSolve : EpiNoSkip<T> {  // x = K^{-1} rhs
  ProjArgs<T> a;
  __device__ double row(int j, double x, double) const { a.x[j] = (T)x; return 0.0; }
  __device__ void block_done(int, double) const {}
};
template <typename T> struct EpiProjTall2 : EpiNoSkip<T> {  // y = A x
  ProjArgs<T> a;
  __device__ double row(int i, double y, double) const { a.y[i] = (T)y; return 0.0; }
  __device__ void block_done(int, double) const {}
};
template <typename T> struct EpiProjWide1 : EpiNoSkip<T> {  // rhs = A c - d
  ProjArgs<T> a;
  __device__ double row(int i, double u, double) const { a.rhs[i] = (T)(u - (double)a.d[i]); return 0.0; }
  __device__ void block_done(int, double) const {}
};
template <typename T> struct EpiProjWideSolve : EpiNoSkip<T> {  // y = d + K^{-1} rhs; rhs <- d - y
  ProjArgs<T> a;
  __device__ double row(int i, double z, double) const {
    const T yv = (T)((double)a.d[i] + z);
    a.y[i] = yv;
    return 0.0;
  }
  __device__ void block_done(int, double) const {}
};
template <typename T> struct EpiProjWide2 : EpiNoSkip<T> {  // x = c + A^T (d - y)
  ProjArgs<T> a;
  __device__ double column(int j, double z, double) const { a.x[j] = (T)((double)a.c[j] + z); return 0.0; }
  __device__ void tile_done(int, double) const {}
};

template <typename T>
__global__ void sub_kernel(const T *a, const T *b, T *out, int len) {  // out = a - b
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) out[i] = a[i] - b[i];
}

// ---------------------------------------------------------------------------
// Geometry and dispatch
// ---------------------------------------------------------------------------
int gemv_t_tile(int elem_size) { return kWave * (16 / elem_size); }

void gemv_t_geometry(int m, int ncols, int elem_size, int *splits, int *rows_per_split, int *ncolp) {
  const int tile = gemv_t_tile(elem_size);
  const int tiles = (int)cdiv(ncols, tile);
  int s = std::max(1, std::min((int)cdiv(m, 16), 1024 / std::max(tiles, 1)));
  // splits shorter than 256 rows cost more in partials and their finish than
  // they gain in parallelism while more than 512 workgroups remain (measured on
  // gfx950: 20000 x 2000 pass 1 29.9 -> 28.7 us; 100000 x 1000 keeps 256 splits)
  while (s > 1 && m / s < 256 && s * tiles > 512) s = (s + 1) / 2;
  int rps = (int)cdiv(m, s);
  rps = (int)round_up(rps, 4);
  s = (int)cdiv(m, rps);
  *splits = s;
  *rows_per_split = rps;
  *ncolp = tiles * tile;
}

// float32 rows of at most 2048 elements: whole rows per wave.  The grid
// targets two workgroups per CU for rows longer than 1024 elements and three
// otherwise (measured best on gfx950: 28 us for 20000 x 2000 at two, 34-36 us
// at 2.5-3), then shrinks so every wave gets the same number of rows (the
// last wave of the grid at most one fewer): a pass ends when its busiest wave
// does.
constexpr int kRowsMaxLd = 2048;
static int rows_grid(int m, int ld) {
  constexpr int kWavesPerBlock = kBlock / kWave;
  const int64_t target = (int64_t)(ld > 1024 ? 2 : 3) * 256 * kWavesPerBlock;
  const int64_t per_wave = cdiv((int64_t)m, target);
  const int64_t waves = cdiv((int64_t)m, per_wave);
  return (int)cdiv(waves, (int64_t)kWavesPerBlock);
}

// Kernel variant and grid of a row-dot pass (A v) over an m x n matrix with
// leading dimension ld: whole rows per wave for float32 rows up to 2048
// elements (NC 16-byte loads per lane), else LDS-staged vectors with 64 or 16
// lanes per row and 1 or 4 rows per lane group.
GemvNShape gemv_n_shape(int m, int n, int ld, int elem_size) {
  GemvNShape sh{};
  if (elem_size == 4 && ld <= kRowsMaxLd) {
    sh.variant = ld <= 256 ? GEMV_N_ROWS1 : ld <= 512 ? GEMV_N_ROWS2 : ld <= 1024 ? GEMV_N_ROWS4 : GEMV_N_ROWS8;
    sh.grid = rows_grid(m, ld);
    return sh;
  }
  const int VN = 16 / elem_size;
  const int vpr = (int)cdiv(n, VN);
  if (vpr >= 128) {
    const int rows1 = gemv_n_rows_per_block<64, 1>();
    if (cdiv(m, rows1) > 2048) {
      sh.variant = GEMV_N_L64R4;
      sh.grid = (int)cdiv(m, gemv_n_rows_per_block<64, 4>());
    } else {
      sh.variant = GEMV_N_L64R1;
      sh.grid = (int)cdiv(m, rows1);
    }
  } else {
    const int rows1 = gemv_n_rows_per_block<16, 1>();
    if (cdiv(m, rows1) > 2048) {
      sh.variant = GEMV_N_L16R4;
      sh.grid = (int)cdiv(m, gemv_n_rows_per_block<16, 4>());
    } else {
      sh.variant = GEMV_N_L16R1;
      sh.grid = (int)cdiv(m, rows1);
    }
  }
  return sh;
}

int gemv_n_blocks(int m, int ncols, int elem_size, int) {
  return gemv_n_shape(m, ncols, (int)round_up(ncols, 64), elem_size).grid;
}

// which: 0 prox (with the previous stop test), 1 first pass over A, 2 solve, 3 second pass over A.
// The one-pass tall iteration (p.fused) has no separate prox launch: part 0 is
// empty, part 1 is the stop test with the first pass where the previous
// iteration's results do not stand (tall_pass1_prox_body) and the finish
// with the x side of the prox step, part 3 the pass that reads A for both
// iterations.
template <typename T>
void launch_iteration_part(const IterArgs<T> &p, int which, int splits, int rps, int ncolp, hipStream_t s) {
  const bool tall = p.m >= p.n;
  switch (which) {
    case 0:
      if (p.fused) break;
      hipLaunchKernelGGL(prox_kernel<T>, dim3(p.nbx + p.nby), dim3(kBlock), 0, s, p);
      break;
    case 1:
      if (p.fused) {
        const dim3 grid((unsigned)cdiv(p.n, gemv_t_tile(sizeof(T))), (unsigned)splits);
        if (p.nt_cols)
          hipLaunchKernelGGL((tall_pass1_prox_kernel<T, true>), grid, dim3(kBlock), 0, s, p, rps, ncolp);
        else
          hipLaunchKernelGGL((tall_pass1_prox_kernel<T, false>), grid, dim3(kBlock), 0, s, p, rps, ncolp);
        hipLaunchKernelGGL(tall_finish_prox_kernel<T>, dim3((unsigned)cdiv(p.n, kFinishCols)), dim3(kBlock), 0, s,
                           p, splits, ncolp);
      } else if (tall) {
        EpiTallPass1<T> e{{p}};
        gemv_t<T, T, 2>(p.A, p.m, p.n, p.ld, p.dy, p.nu, splits, rps, p.part, ncolp, e, s, p.nt_cols);
      } else {
        EpiWidePass1<T> e{{p}};
        gemv_n<T, T, 2>(p.A, p.m, p.n, p.ld, p.cx, p.xh, e, s, p.nt_rows);
      }
      break;
    case 2:
      if (!p.Kinv) break;  // no factor (a context set up for CGLS): nothing to solve with
      if (tall) {
        EpiTallSolve<T> e{{p}};
        gemv_n<T, T, 1>(p.Kinv, p.q, p.q, p.ldk, p.rhs, p.rhs, e, s);
      } else {
        EpiWideSolve<T> e{{p}};
        gemv_n<T, T, 1>(p.Kinv, p.q, p.q, p.ldk, p.rhs, p.rhs, e, s);
      }
      break;
    default:
      if (p.fused) {
        if constexpr (std::is_same<T, float>::value) {
          if (p.nt_rows) launch_one_pass_nt<true>(p, ncolp, s);
          else launch_one_pass_nt<false>(p, ncolp, s);
        }
      } else if (tall) {
        EpiTallPass2<T> e{{p}};
        gemv_n<T, T, 2>(p.A, p.m, p.n, p.ld, p.x, p.xh, e, s, p.nt_rows);
      } else {
        EpiWidePass2<T> e{{p}};
        gemv_t<T, T, 2>(p.A, p.m, p.n, p.ld, p.yt, p.nu, splits, rps, p.part, ncolp, e, s, p.nt_cols);
      }
      break;
  }
}

template <typename T>
void launch_iteration(const IterArgs<T> &p, int splits, int rps, int ncolp, hipStream_t s) {
  for (int w = 0; w < 4; ++w) launch_iteration_part<T>(p, w, splits, rps, ncolp, s);
}

template <typename T>
void launch_iteration_gap(const IterArgs<T> &p, int splits, int rps, int ncolp, hipStream_t s) {
  launch_iteration_part<T>(p, 0, splits, rps, ncolp, s);
  launch_gap_check<T>(p, s);
  for (int w = 1; w < 4; ++w) launch_iteration_part<T>(p, w, splits, rps, ncolp, s);
}

template <typename T> void launch_control_preview(const IterArgs<T> &p, int par, hipStream_t s) {
  hipLaunchKernelGGL(control_preview_kernel<T>, dim3(1), dim3(kBlock), 0, s, p, par);
}

template <typename T>
void launch_project(const IterArgs<T> &p, int splits, int rps, int ncolp, const T *c, const T *d, T *x,
                    T *y, hipStream_t s) {
  ProjArgs<T> a{c, d, x, y, p.rhs};
  if (p.m >= p.n) {
    EpiProjTall1<T> e1; e1.a = a;
    gemv_t<T, T, 1>(p.A, p.m, p.n, p.ld, d, d, splits, rps, p.part, ncolp, e1, s);
    EpiProjTallSolve<T> e2; e2.a = a;
    gemv_n<T, T, 1>(p.Kinv, p.q, p.q, p.ldk, p.rhs, p.rhs, e2, s);
    EpiProjTall2<T> e3; e3.a = a;
    gemv_n<T, T, 1>(p.A, p.m, p.n, p.ld, x, x, e3, s);
  } else {
    EpiProjWide1<T> e1; e1.a = a;
    gemv_n<T, T, 1>(p.A, p.m, p.n, p.ld, c, c, e1, s);
    EpiProjWideSolve<T> e2; e2.a = a;
    gemv_n<T, T, 1>(p.Kinv, p.q, p.q, p.ldk, p.rhs, p.rhs, e2, s);
    // rhs <- d - y, then x = c + A^T rhs
    hipLaunchKernelGGL(sub_kernel<T>, dim3(cdiv(p.m, kBlock)), dim3(kBlock), 0, s, d, (const T *)y, p.rhs, p.m);
    EpiProjWide2<T> e3; e3.a = a;
    gemv_t<T, T, 1>(p.A, p.m, p.n, p.ld, p.rhs, p.rhs, splits, rps, p.part, ncolp, e3, s);
  }
}

// ---------------------------------------------------------------------------
// Warm start from (x0, nu0) in the original variables: x = E^-1 x0 and
// y = A^ x (a point of the graph); y~ = -(D^-1 nu0) / rho0 (the scaled dual
// the prox step returns when it leaves y unchanged); x~ = -A^T y~ (the
// relation every projection restores).  With only one of them, the other is
// estimated by warm_estimate_kernel: x0 only -> y~ = prox_f^(y) - y, then
// x~ = -A^T y~; nu0 only -> x = prox_g^(-x~), then y = A^ x.
// ---------------------------------------------------------------------------
template <typename T> struct EpiWarmY : EpiNoSkip<T> {  // y = A x
  T *y;
  __device__ double row(int i, double v, double) const { y[i] = (T)v; return 0.0; }
  __device__ void block_done(int, double) const {}
};
template <typename T> struct EpiWarmXt : EpiNoSkip<T> {  // x~ = -A^T y~
  T *xt;
  __device__ double column(int j, double v, double) const { xt[j] = (T)(-v); return 0.0; }
  __device__ void tile_done(int, double) const {}
};

template <typename T>
void launch_warm_start(const IterArgs<T> &p, int splits, int rps, int ncolp, const double *D, const double *E,
                       double rho0, const T *x0, const T *nu0, hipStream_t s) {
  if (x0) {
    hipLaunchKernelGGL(warm_scale_kernel<T>, dim3(cdiv(p.n, kBlock)), dim3(kBlock), 0, s, x0, E, true, 1.0, p.n,
                       p.x);
    EpiWarmY<T> e;
    e.y = p.y;
    gemv_n<T, T, 1>(p.A, p.m, p.n, p.ld, (const T *)p.x, (const T *)p.x, e, s);
  }
  if (nu0) {
    hipLaunchKernelGGL(warm_scale_kernel<T>, dim3(cdiv(p.m, kBlock)), dim3(kBlock), 0, s, nu0, D, true,
                       -1.0 / rho0, p.m, p.yt);
  } else if (x0) {
    hipLaunchKernelGGL(warm_estimate_kernel<T>, dim3(cdiv(p.m, kBlock)), dim3(kBlock), 0, s, p.f, (const T *)p.y,
                       p.yt, p.m, (T)rho0, 0);
  }
  if (nu0 || x0) {
    EpiWarmXt<T> e;
    e.xt = p.xt;
    gemv_t<T, T, 1>(p.A, p.m, p.n, p.ld, (const T *)p.yt, (const T *)p.yt, splits, rps, p.part, ncolp, e, s);
  }
  if (nu0 && !x0) {
    hipLaunchKernelGGL(warm_estimate_kernel<T>, dim3(cdiv(p.n, kBlock)), dim3(kBlock), 0, s, p.g, (const T *)p.xt,
                       p.x, p.n, (T)rho0, 1);
    EpiWarmY<T> e;
    e.y = p.y;
    gemv_n<T, T, 1>(p.A, p.m, p.n, p.ld, (const T *)p.x, (const T *)p.x, e, s);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void scale_fn_kernel(const uint8_t *h, const double *a, const double *b,
                                                          const double *c, const double *d, const double *e,
                                                          const double *scale, bool divide, int len, uint8_t *oh,
                                                          T *oa, T *ob, T *oc, T *od, T *oe) {
  scale_fn_body<T>(hw_block(), h, a, b, c, d, e, scale, divide, len, oh, oa, ob, oc, od, oe);
}

template <typename T>
void launch_scale_fn(const uint8_t *h, const double *a, const double *b, const double *c, const double *d,
                     const double *e, const double *scale, bool divide, int len, uint8_t *oh, T *oa,
                     T *ob, T *oc, T *od, T *oe, hipStream_t s) {
  hipLaunchKernelGGL(scale_fn_kernel<T>, dim3(cdiv(len, kBlock)), dim3(kBlock), 0, s, h, a, b, c, d, e,
                     scale, divide, len, oh, oa, ob, oc, od, oe);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void unscale_kernel(
    IterArgs<T> p, const double *D, const double *E, const uint8_t *fh, const double *fa,
    const double *fb, const double *fc, const double *fd, const double *fe, const uint8_t *gh,
    const double *ga, const double *gb, const double *gc, const double *gd, const double *ge, T *xo,
    T *yo, T *muo, T *nuo, double *slots, double *obj, unsigned *cnt, int from_state, double rho) {
  unscale_body<T>(hw_block(), p, D, E, fh, fa, fb, fc, fd, fe, gh, ga, gb, gc, gd, ge, xo, yo, muo, nuo, slots, obj,
                  cnt, from_state, rho);
}

template <typename T>
void launch_unscale(const IterArgs<T> &p, const double *D, const double *E, const uint8_t *fh0,
                    const double *fa0, const double *fb0, const double *fc0, const double *fd0,
                    const double *fe0, const uint8_t *gh0, const double *ga0, const double *gb0,
                    const double *gc0, const double *gd0, const double *ge0, T *xo, T *yo, T *muo,
                    T *nuo, double *obj_slots, double *obj_out, unsigned *cnt, int from_state, double rho,
                    hipStream_t s) {
  hipLaunchKernelGGL(unscale_kernel<T>, dim3(p.nbx + p.nby), dim3(kBlock), 0, s, p, D, E, fh0, fa0, fb0,
                     fc0, fd0, fe0, gh0, ga0, gb0, gc0, gd0, ge0, xo, yo, muo, nuo, obj_slots, obj_out, cnt,
                     from_state, rho);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void gap_check_kernel(IterArgs<T> p) {
  gap_check_body<T>(p);
}

template <typename T> void launch_gap_check(const IterArgs<T> &p, hipStream_t s) {
  hipLaunchKernelGGL(gap_check_kernel<T>, dim3(1), dim3(kBlock), 0, s, p);
}

// ---------------------------------------------------------------------------
// Elementwise prox evaluation (primitive)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void prox_eval_kernel(const uint8_t *h, const T *a, const T *b, const T *c, const T *d,
                                 const T *e, T rho, const T *v, T *out, int len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) out[i] = prox_param<T>(h[i], a[i], b[i], c[i], d[i], e[i], v[i], rho);
}

template <typename T>
void launch_prox_eval(const uint8_t *h, const T *a, const T *b, const T *c, const T *d, const T *e,
                      double rho, const T *v, T *out, int len, hipStream_t s) {
  hipLaunchKernelGGL(prox_eval_kernel<T>, dim3(cdiv(len, kBlock)), dim3(kBlock), 0, s, h, a, b, c, d, e,
                     (T)rho, v, out, len);
}

#define POGS_INST(T)                                                                                   \
  template void launch_iteration<T>(const IterArgs<T> &, int, int, int, hipStream_t);                  \
  template void launch_iteration_gap<T>(const IterArgs<T> &, int, int, int, hipStream_t);              \
  template void launch_iteration_part<T>(const IterArgs<T> &, int, int, int, int, hipStream_t);        \
  template void launch_control_preview<T>(const IterArgs<T> &, int, hipStream_t);                      \
  template void launch_project<T>(const IterArgs<T> &, int, int, int, const T *, const T *, T *, T *,  \
                                  hipStream_t);                                                        \
  template void launch_warm_start<T>(const IterArgs<T> &, int, int, int, const double *, const double *, \
                                     double, const T *, const T *, hipStream_t);                         \
  template void launch_scale_fn<T>(const uint8_t *, const double *, const double *, const double *,    \
                                   const double *, const double *, const double *, bool, int,          \
                                   uint8_t *, T *, T *, T *, T *, T *, hipStream_t);                   \
  template void launch_unscale<T>(const IterArgs<T> &, const double *, const double *,                 \
                                  const uint8_t *, const double *, const double *, const double *,     \
                                  const double *, const double *, const uint8_t *, const double *,     \
                                  const double *, const double *, const double *, const double *, T *, \
                                  T *, T *, T *, double *, double *, unsigned *, int, double,          \
                                  hipStream_t);                                                        \
  template void launch_gap_check<T>(const IterArgs<T> &, hipStream_t);                                 \
  template void launch_prox_eval<T>(const uint8_t *, const T *, const T *, const T *, const T *,       \
                                    const T *, double, const T *, T *, int, hipStream_t);
POGS_INST(float)
POGS_INST(double)
#undef POGS_INST

}  // namespace pogs
