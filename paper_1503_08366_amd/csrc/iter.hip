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
#include "gemv.hpp"
#include "internal.hpp"
#include "prox.hpp"

namespace pogs {

// ---------------------------------------------------------------------------
// Stopping test and adaptive penalty for the iteration whose partial sums are
// in the slots (Section 3.4, Algorithm 3), in two parts so the slot loads can
// be issued together with the caller's other loads:
//   control_partials: this thread's share of the four slot sums (parity spar);
//   control_apply:    fixed-order block sums, then thread 0 updates `st`
//                     (LDS), valid in every thread after the call.
// ---------------------------------------------------------------------------
template <typename T>
__device__ inline void control_partials(const IterArgs<T> &p, int spar, double part[4]) {
  const double *s_mu = p.s_mu + (size_t)spar * p.nbx;
  const double *s_yh = p.s_yh + (size_t)spar * p.nby;
  part[0] = part[1] = part[2] = part[3] = 0.0;
  for (int i = threadIdx.x; i < p.nbx; i += blockDim.x) part[0] += s_mu[i];
  for (int i = threadIdx.x; i < p.nby; i += blockDim.x) part[1] += s_yh[i];
  for (int i = threadIdx.x; i < p.n_pri; i += blockDim.x) part[2] += p.s_pri[i];
  for (int i = threadIdx.x; i < p.n_dual; i += blockDim.x) part[3] += p.s_dual[i];
}

// Four block-wide sums at once (one barrier pair); results valid in thread 0.
// Fixed order: wave shuffle tree, then the waves in index order.
__device__ inline void block_sum4(double v[4], double *scratch /* 4 * waves */) {
  const int nw = blockDim.x / kWave, w = threadIdx.x / kWave;
#pragma unroll
  for (int c = 0; c < 4; ++c) v[c] = wave_sum(v[c]);
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) scratch[c * nw + w] = v[c];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      double t = 0.0;
      for (int i = 0; i < nw; ++i) t += scratch[c * nw + i];
      v[c] = t;
    }
}

template <typename T>
__device__ void control_apply(const IterArgs<T> &p, double part[4], CtrlState &st, double *lds) {
  block_sum4(part, lds);
  if (threadIdx.x == 0) {
    const Ctrl &q = *p.ctrl;
    const double mu2 = part[0], yh2 = part[1], pri2 = part[2], dual2 = part[3];
    const double r_pri = sqrt(pri2), r_dual = sqrt(dual2);
    const double eps_pri = q.eps_abs + q.eps_rel * sqrt(yh2);
    const double eps_dual = q.eps_abs + q.eps_rel * sqrt(mu2);
    st.r_pri = r_pri;
    st.r_dual = r_dual;
    st.eps_pri = eps_pri;
    st.eps_dual = eps_dual;
    const int k = st.k;
    double rescale = 1.0;
    int done = 0;
    if (!isfinite(r_pri) || !isfinite(r_dual)) {
      done = 1 + POGS_NUMERICAL;
    } else if (r_pri < eps_pri && r_dual < eps_dual) {
      done = 1 + POGS_CONVERGED;
    } else {
      if (q.adaptive) {
        const double rho = st.rho;
        double rho_new = rho;
        if (r_dual < eps_dual && q.tau * k > st.l) {
          rho_new = q.delta * rho;
          st.u = k;
        } else if (r_pri < eps_pri && q.tau * k > st.u) {
          rho_new = rho / q.delta;
          st.l = k;
        }
        if (rho_new != rho) {
          rescale = rho / rho_new;
          st.rho = rho_new;
        }
      }
      if (k + 1 >= q.max_iter) done = 1 + POGS_MAXITER;
    }
    st.rescale = rescale;
    st.k = k + 1;
    st.done = done;
    st.pending = 0;
  }
  __syncthreads();
}

// Stop test of the last iteration of a launch sequence (parity `par`), so the
// host sees the flag; the next prox step recomputes the same state (a pure
// function of the stored state and the partial sums).
template <typename T>
__global__ __launch_bounds__(kBlock) void control_preview_kernel(IterArgs<T> p, int par) {
  __shared__ double bs[4 * (kBlock / kWave)];
  __shared__ CtrlState st;
  if (threadIdx.x == 0) st = p.ctrl->st[par];
  double part[4];
  control_partials(p, par, part);
  __syncthreads();
  if (!st.done && st.pending) control_apply(p, part, st, bs);
  if (threadIdx.x == 0) p.ctrl->st[1 - par] = st;
}

// ---------------------------------------------------------------------------
// 1. prox step (runs the previous iteration's stop test first)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void prox_kernel(IterArgs<T> p) {
  __shared__ double bs[4 * (kBlock / kWave)];
  __shared__ CtrlState st;
  const int par = p.par;
  const bool xs = (int)blockIdx.x < p.nbx;
  const int blk = xs ? blockIdx.x : blockIdx.x - p.nbx;
  const int i = blk * kBlock + threadIdx.x;
  const int len = xs ? p.n : p.m;
  // every load that does not depend on the control state goes out first
  if (threadIdx.x == 0) st = p.ctrl->st[1 - par];
  double part[4];
  control_partials(p, 1 - par, part);
  const FnDev<T> &F = xs ? p.g : p.f;
  T *v = xs ? p.x : p.y;
  T *vt = xs ? p.xt : p.yt;
  T vi = T(0), vti = T(0), fa = T(0), fb = T(0), fc = T(0), fd = T(0), fe = T(0);
  int fh = 0;
  if (i < len) {
    vi = v[i];
    vti = vt[i];
    fh = F.h[i];
    fa = F.a[i];
    fb = F.b[i];
    fc = F.c[i];
    fd = F.d[i];
    fe = F.e[i];
  }
  __syncthreads();
  if (!st.done && st.pending) control_apply(p, part, st, bs);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    CtrlState out = st;
    out.pending = st.done ? 0 : 1;
    p.ctrl->st[par] = out;
  }
  if (st.done) return;
  const T rho = (T)st.rho;
  const T resc = (T)st.rescale;
  const T alpha = (T)p.ctrl->alpha;
  double contrib = 0.0;
  if (i < len) {
    if (resc != T(1)) {
      vti *= resc;
      vt[i] = vti;
    }
    const T arg = vi - vti;
    const T h = prox_param<T>(fh, fa, fb, fc, fd, fe, arg, rho);
    const T dual = -rho * (h - arg);
    const T rel = alpha * h + (T(1) - alpha) * vi;
    (xs ? p.xh : p.yh)[i] = h;
    (xs ? p.mu : p.nu)[i] = dual;
    (xs ? p.cx : p.dy)[i] = rel + vti;
    contrib = xs ? (double)dual * (double)dual : (double)h * (double)h;
  }
  const double s = block_sum(contrib, bs);
  if (threadIdx.x == 0) (xs ? p.s_mu + (size_t)par * p.nbx : p.s_yh + (size_t)par * p.nby)[blk] = s;
}

// ---------------------------------------------------------------------------
// Epilogues
// ---------------------------------------------------------------------------
template <typename T> struct EpiBase {
  IterArgs<T> p;
  __device__ bool skip() const { return p.ctrl->st[p.par].done != 0; }
};

// m >= n, pass 1: [w, s] = A^T [d, nu_h]
template <typename T> struct EpiTallPass1 : EpiBase<T> {
  __device__ double column(int j, double w, double s) const {
    const IterArgs<T> &p = this->p;
    p.rhs[j] = (T)((double)p.cx[j] + w);
    const double r = s + (double)p.mu[j];
    return r * r;
  }
  __device__ void tile_done(int tile, double v) const { this->p.s_dual[tile] = v; }
};

// m >= n, solve: x = K^{-1} rhs
template <typename T> struct EpiTallSolve : EpiBase<T> {
  __device__ double row(int j, double x, double) const {
    const IterArgs<T> &p = this->p;
    const T xv = (T)x;
    p.x[j] = xv;
    p.xt[j] = p.cx[j] - xv;
    return 0.0;
  }
  __device__ void block_done(int, double) const {}
};

// m >= n, pass 2: [y, t] = A [x, x_h]; then the stopping test
template <typename T> struct EpiTallPass2 : EpiBase<T> {
  __device__ double row(int i, double y, double t) const {
    const IterArgs<T> &p = this->p;
    const T yv = (T)y;
    p.y[i] = yv;
    p.yt[i] = p.dy[i] - yv;
    const double r = t - (double)p.yh[i];
    return r * r;
  }
  __device__ void block_done(int b, double v) const { this->p.s_pri[b] = v; }
};

// m < n, pass 1: [u, t] = A [c, x_h]
template <typename T> struct EpiWidePass1 : EpiBase<T> {
  __device__ double row(int i, double u, double t) const {
    const IterArgs<T> &p = this->p;
    p.rhs[i] = (T)(u - (double)p.dy[i]);
    const double r = t - (double)p.yh[i];
    return r * r;
  }
  __device__ void block_done(int b, double v) const { this->p.s_pri[b] = v; }
};

// m < n, solve: y = d + K^{-1} rhs, y~ = d - y
template <typename T> struct EpiWideSolve : EpiBase<T> {
  __device__ double row(int i, double z, double) const {
    const IterArgs<T> &p = this->p;
    const T yv = (T)((double)p.dy[i] + z);
    p.y[i] = yv;
    p.yt[i] = p.dy[i] - yv;
    return 0.0;
  }
  __device__ void block_done(int, double) const {}
};

// m < n, pass 2: [z, s] = A^T [y~, nu_h]; x = c + z, x~ = c - x; then stop test
template <typename T> struct EpiWidePass2 : EpiBase<T> {
  __device__ double column(int j, double z, double s) const {
    const IterArgs<T> &p = this->p;
    const T xv = (T)((double)p.cx[j] + z);
    p.x[j] = xv;
    p.xt[j] = p.cx[j] - xv;
    const double r = s + (double)p.mu[j];
    return r * r;
  }
  __device__ void tile_done(int tile, double v) const { this->p.s_dual[tile] = v; }
};

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
  int rps = (int)cdiv(m, s);
  rps = (int)round_up(rps, 4);
  s = (int)cdiv(m, rps);
  *splits = s;
  *rows_per_split = rps;
  *ncolp = tiles * tile;
}

template <typename T, typename TV, int NRHS, class Epi>
static void gemv_t(const T *A, int m, int n, int ld, const TV *v0, const TV *v1, int splits, int rps,
                   double *part, int ncolp, const Epi &epi, hipStream_t s) {
  const int tile = gemv_t_tile(sizeof(T));
  const int tiles = (int)cdiv(n, tile);
  dim3 grid(tiles, splits);
  hipLaunchKernelGGL((gemv_t_kernel<T, TV, NRHS, false, Epi>), grid, dim3(kBlock), 0, s, A, m, n, ld, v0, v1, rps,
                     part, ncolp, epi);
  hipLaunchKernelGGL((gemv_t_finish_kernel<NRHS, Epi>), dim3(cdiv(n, kFinishCols)), dim3(kBlock), 0, s, n, splits,
                     (const double *)part, ncolp, epi);
}

// float32 rows of at most 2048 elements: whole rows per wave, the grid one
// round of resident workgroups (four per CU up to 1024 columns, three above;
// the kernel's register budget guarantees that residency on 256 CUs).
constexpr int kRowsMaxLd = 2048;
static int rows_grid(int m, int ld) {
  return (int)std::min<int64_t>(cdiv(m, kBlock / kWave), (ld > 1024 ? 3 : 4) * 256);
}

template <int NRHS, int NC, class Epi>
static void launch_rows(const float *A, int m, int n, int ld, const float *v0, const float *v1, const Epi &epi,
                        hipStream_t s) {
  hipLaunchKernelGGL((gemv_n_rows_kernel<NRHS, NC, Epi>), dim3(rows_grid(m, ld)), dim3(kBlock), 0, s, A, m, n, ld,
                     v0, v1, epi);
}

// Pick the kernel and its shape from the row length and row count.
template <typename T, typename TV, int NRHS, class Epi>
static void gemv_n(const T *A, int m, int n, int ld, const TV *v0, const TV *v1, const Epi &epi, hipStream_t s,
                   int *nblocks_out = nullptr) {
  if constexpr (sizeof(T) == 4 && sizeof(TV) == 4) {
    if (ld <= kRowsMaxLd) {
      const float *Af = (const float *)A, *x0 = (const float *)v0, *x1 = (const float *)v1;
      if (ld <= 256) launch_rows<NRHS, 1>(Af, m, n, ld, x0, x1, epi, s);
      else if (ld <= 512) launch_rows<NRHS, 2>(Af, m, n, ld, x0, x1, epi, s);
      else if (ld <= 1024) launch_rows<NRHS, 4>(Af, m, n, ld, x0, x1, epi, s);
      else launch_rows<NRHS, 8>(Af, m, n, ld, x0, x1, epi, s);
      if (nblocks_out) *nblocks_out = rows_grid(m, ld);
      return;
    }
  }
  constexpr int VN = Vec16<T>::N;
  const int vpr = (int)cdiv(n, VN);
  const bool wide_rows = vpr >= 128;
  int nb;
  if (wide_rows) {
    const int rows1 = gemv_n_rows_per_block<64, 1>();
    if (cdiv(m, rows1) > 2048) {
      nb = (int)cdiv(m, gemv_n_rows_per_block<64, 4>());
      hipLaunchKernelGGL((gemv_n_kernel<T, TV, NRHS, false, 64, 4, Epi>), dim3(nb), dim3(kBlock), 0, s,
                         A, m, n, ld, v0, v1, epi);
    } else {
      nb = (int)cdiv(m, rows1);
      hipLaunchKernelGGL((gemv_n_kernel<T, TV, NRHS, false, 64, 1, Epi>), dim3(nb), dim3(kBlock), 0, s,
                         A, m, n, ld, v0, v1, epi);
    }
  } else {
    const int rows1 = gemv_n_rows_per_block<16, 1>();
    if (cdiv(m, rows1) > 2048) {
      nb = (int)cdiv(m, gemv_n_rows_per_block<16, 4>());
      hipLaunchKernelGGL((gemv_n_kernel<T, TV, NRHS, false, 16, 4, Epi>), dim3(nb), dim3(kBlock), 0, s,
                         A, m, n, ld, v0, v1, epi);
    } else {
      nb = (int)cdiv(m, rows1);
      hipLaunchKernelGGL((gemv_n_kernel<T, TV, NRHS, false, 16, 1, Epi>), dim3(nb), dim3(kBlock), 0, s,
                         A, m, n, ld, v0, v1, epi);
    }
  }
  if (nblocks_out) *nblocks_out = nb;
}

int gemv_n_blocks(int m, int ncols, int elem_size, int) {
  if (elem_size == 4 && round_up(ncols, 64) <= kRowsMaxLd) return rows_grid(m, (int)round_up(ncols, 64));
  const int VN = 16 / elem_size;
  const int vpr = (int)cdiv(ncols, VN);
  if (vpr >= 128) {
    const int rows1 = gemv_n_rows_per_block<64, 1>();
    return cdiv(m, rows1) > 2048 ? (int)cdiv(m, gemv_n_rows_per_block<64, 4>()) : (int)cdiv(m, rows1);
  }
  const int rows1 = gemv_n_rows_per_block<16, 1>();
  return cdiv(m, rows1) > 2048 ? (int)cdiv(m, gemv_n_rows_per_block<16, 4>()) : (int)cdiv(m, rows1);
}

// which: 0 prox (with the previous stop test), 1 first pass over A, 2 solve, 3 second pass over A.
template <typename T>
void launch_iteration_part(const IterArgs<T> &p, int which, int splits, int rps, int ncolp, hipStream_t s) {
  const bool tall = p.m >= p.n;
  switch (which) {
    case 0:
      hipLaunchKernelGGL(prox_kernel<T>, dim3(p.nbx + p.nby), dim3(kBlock), 0, s, p);
      break;
    case 1:
      if (tall) {
        EpiTallPass1<T> e{{p}};
        gemv_t<T, T, 2>(p.A, p.m, p.n, p.ld, p.dy, p.nu, splits, rps, p.part, ncolp, e, s);
      } else {
        EpiWidePass1<T> e{{p}};
        gemv_n<T, T, 2>(p.A, p.m, p.n, p.ld, p.cx, p.xh, e, s);
      }
      break;
    case 2:
      if (tall) {
        EpiTallSolve<T> e{{p}};
        gemv_n<T, T, 1>(p.Kinv, p.q, p.q, p.ldk, p.rhs, p.rhs, e, s);
      } else {
        EpiWideSolve<T> e{{p}};
        gemv_n<T, T, 1>(p.Kinv, p.q, p.q, p.ldk, p.rhs, p.rhs, e, s);
      }
      break;
    default:
      if (tall) {
        EpiTallPass2<T> e{{p}};
        gemv_n<T, T, 2>(p.A, p.m, p.n, p.ld, p.x, p.xh, e, s);
      } else {
        EpiWidePass2<T> e{{p}};
        gemv_t<T, T, 2>(p.A, p.m, p.n, p.ld, p.yt, p.nu, splits, rps, p.part, ncolp, e, s);
      }
      break;
  }
}

template <typename T>
void launch_iteration(const IterArgs<T> &p, int splits, int rps, int ncolp, hipStream_t s) {
  for (int w = 0; w < 4; ++w) launch_iteration_part<T>(p, w, splits, rps, ncolp, s);
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
// Function parameters for the pre-conditioned problem (Section 4.1):
//   f^(y) = f(y / D):  a/D, b, c, d/D, e/D^2      (divide = true, scale = D)
//   g^(x) = g(E x):    a E, b, c, d E, e E^2      (divide = false, scale = E)
// Inputs are float64 per-element arrays; outputs in the iteration type.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void scale_fn_kernel(const uint8_t *h, const double *a, const double *b, const double *c,
                                const double *d, const double *e, const double *scale, bool divide,
                                int len, uint8_t *oh, T *oa, T *ob, T *oc, T *od, T *oe) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  const double s = scale ? (divide ? 1.0 / scale[i] : scale[i]) : 1.0;
  oh[i] = h[i];
  oa[i] = (T)(a[i] * s);
  ob[i] = (T)b[i];
  oc[i] = (T)c[i];
  od[i] = (T)(d[i] * s);
  oe[i] = (T)(e[i] * s * s);
}

template <typename T>
void launch_scale_fn(const uint8_t *h, const double *a, const double *b, const double *c, const double *d,
                     const double *e, const double *scale, bool divide, int len, uint8_t *oh, T *oa,
                     T *ob, T *oc, T *od, T *oe, hipStream_t s) {
  hipLaunchKernelGGL(scale_fn_kernel<T>, dim3(cdiv(len, kBlock)), dim3(kBlock), 0, s, h, a, b, c, d, e,
                     scale, divide, len, oh, oa, ob, oc, od, oe);
}

// ---------------------------------------------------------------------------
// Return the half-step tuple in the original variables (Section 5):
//   x = E x_h, y = y_h / D, mu = mu_h / E, nu = D nu_h,
// and the objective f(y) + g(x) with the unscaled parameters.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void unscale_kernel(
    IterArgs<T> p, const double *D, const double *E, const uint8_t *fh, const double *fa,
    const double *fb, const double *fc, const double *fd, const double *fe, const uint8_t *gh,
    const double *ga, const double *gb, const double *gc, const double *gd, const double *ge, T *xo,
    T *yo, T *muo, T *nuo, double *slots, double *obj, unsigned *cnt) {
  __shared__ double bs[kBlock / kWave];
  __shared__ int flag;
  const bool xs = (int)blockIdx.x < p.nbx;
  const int blk = xs ? blockIdx.x : blockIdx.x - p.nbx;
  const int i = blk * kBlock + threadIdx.x;
  double contrib = 0.0;
  if (xs && i < p.n) {
    const double x = E[i] * (double)p.xh[i];
    if (xo) xo[i] = (T)x;
    if (muo) muo[i] = (T)((double)p.mu[i] / E[i]);
    contrib = fn_value(gh[i], ga[i], gb[i], gc[i], gd[i], ge[i], x);
  } else if (!xs && i < p.m) {
    const double y = (double)p.yh[i] / D[i];
    if (yo) yo[i] = (T)y;
    if (nuo) nuo[i] = (T)(D[i] * (double)p.nu[i]);
    contrib = fn_value(fh[i], fa[i], fb[i], fc[i], fd[i], fe[i], y);
  }
  const double s = block_sum(contrib, bs);
  if (threadIdx.x == 0) slots[blockIdx.x] = s;
  if (arrive_last(cnt, gridDim.x, &flag)) {
    double t = 0.0;
    for (int j = threadIdx.x; j < (int)gridDim.x; j += blockDim.x) t += load_agent(slots + j);
    const double tot = block_sum(t, bs);
    if (threadIdx.x == 0) *obj = tot;
  }
}

template <typename T>
void launch_unscale(const IterArgs<T> &p, const double *D, const double *E, const uint8_t *fh0,
                    const double *fa0, const double *fb0, const double *fc0, const double *fd0,
                    const double *fe0, const uint8_t *gh0, const double *ga0, const double *gb0,
                    const double *gc0, const double *gd0, const double *ge0, T *xo, T *yo, T *muo,
                    T *nuo, double *obj_slots, double *obj_out, unsigned *cnt, hipStream_t s) {
  hipLaunchKernelGGL(unscale_kernel<T>, dim3(p.nbx + p.nby), dim3(kBlock), 0, s, p, D, E, fh0, fa0, fb0,
                     fc0, fd0, fe0, gh0, ga0, gb0, gc0, gd0, ge0, xo, yo, muo, nuo, obj_slots, obj_out, cnt);
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
  template void launch_iteration_part<T>(const IterArgs<T> &, int, int, int, int, hipStream_t);        \
  template void launch_control_preview<T>(const IterArgs<T> &, int, hipStream_t);                      \
  template void launch_project<T>(const IterArgs<T> &, int, int, int, const T *, const T *, T *, T *,  \
                                  hipStream_t);                                                        \
  template void launch_scale_fn<T>(const uint8_t *, const double *, const double *, const double *,    \
                                   const double *, const double *, const double *, bool, int,          \
                                   uint8_t *, T *, T *, T *, T *, T *, hipStream_t);                   \
  template void launch_unscale<T>(const IterArgs<T> &, const double *, const double *,                 \
                                  const uint8_t *, const double *, const double *, const double *,     \
                                  const double *, const double *, const uint8_t *, const double *,     \
                                  const double *, const double *, const double *, const double *, T *, \
                                  T *, T *, T *, double *, double *, unsigned *, hipStream_t);         \
  template void launch_prox_eval<T>(const uint8_t *, const T *, const T *, const T *, const T *,       \
                                    const T *, double, const T *, T *, int, hipStream_t);
POGS_INST(float)
POGS_INST(double)
#undef POGS_INST

}  // namespace pogs
