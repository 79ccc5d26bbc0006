// Device-side pieces of one ADMM iteration shared by the single-problem
// launches (iter.hip) and the grouped launches over many problems
// (group.hip): the stop test and Algorithm 3, the prox step, the epilogues
// of the passes over A, the pre-conditioned function parameters and the
// return to the original variables.  Every body takes its block
// coordinates explicitly (Blk).
#pragma once

#include "gemv.hpp"
#include "internal.hpp"
#include "gap.hpp"
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
    } else if (!q.stop_gap && r_pri < eps_pri && r_dual < eps_dual) {
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
__device__ __forceinline__ void control_preview_body(const IterArgs<T> &p, int par) {
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
// With CG (the CGLS projection) the state is read as that projection leaves
// it: x~ = c - x, y = d - r1, y~ = r1 (r1 kept in yt), and x is set to the
// half step x_h, where the next projection starts.
template <typename T, bool CG = false>
__device__ __forceinline__ void prox_body(const Blk &b, const IterArgs<T> &p) {
  __shared__ double bs[4 * (kBlock / kWave)];
  __shared__ CtrlState st;
  const int par = p.par;
  const bool xs = b.x < p.nbx;
  const int blk = xs ? b.x : b.x - p.nbx;
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
    if constexpr (CG) {
      if (xs) {
        vi = p.x[i];
        vti = p.cx[i] - vi;
      } else {
        vti = p.yt[i];
        vi = p.dy[i] - vti;
      }
    } else {
      vi = v[i];
      vti = vt[i];
    }
    fh = F.h[i];
    fa = F.a[i];
    fb = F.b[i];
    fc = F.c[i];
    fd = F.d[i];
    fe = F.e[i];
  }
  __syncthreads();
  if (!st.done && st.pending) control_apply(p, part, st, bs);
  if (b.x == 0 && threadIdx.x == 0) {
    CtrlState out = st;
    out.pending = st.done ? 0 : 1;
    p.ctrl->st[par] = out;
  }
  if (st.done) return;
  const T rho = (T)st.rho;
  const T resc = (T)st.rescale;
  const T alpha = (T)p.ctrl->alpha;
  const bool gap = !CG && p.ctrl->stop_gap;
  double contrib = 0.0, gobj = 0.0, gconj = 0.0;
  if (i < len) {
    if (resc != T(1)) {
      vti *= resc;
      if constexpr (!CG) vt[i] = vti;
    }
    if (gap) {
      // the state is primal and dual feasible: value at (x, y), conjugate at
      // (mu, nu) = (-rho x~, -rho y~)
      gobj = fn_value_strict(fh, fa, fb, fc, fd, fe, (double)vi);
      gconj = fn_conj_value(fh, fa, fb, fc, fd, fe, -(double)st.rho * (double)vti);
    }
    const T arg = vi - vti;
    const T h = prox_param<T>(fh, fa, fb, fc, fd, fe, arg, rho);
    const T dual = -rho * (h - arg);
    const T rel = alpha * h + (T(1) - alpha) * vi;
    if (xs) {
      p.xh[i] = h;
      p.mu[i] = dual;
      p.cx[i] = rel + vti;
      if constexpr (CG) p.x[i] = h;
    } else {
      p.yh[i] = h;
      p.nu[i] = dual;
      p.dy[i] = rel + vti;
    }
    contrib = xs ? (double)dual * (double)dual : (double)h * (double)h;
  }
  const double s = block_sum(contrib, bs);
  if (threadIdx.x == 0) {
    if (xs) p.s_mu[(size_t)par * p.nbx + blk] = s;
    else p.s_yh[(size_t)par * p.nby + blk] = s;
  }
  if (gap) {
    const double so = block_sum(gobj, bs);
    const double sc = block_sum(gconj, bs);
    if (threadIdx.x == 0) {
      p.s_gobj[b.x] = so;
      p.s_gconj[b.x] = sc;
    }
  }
}

// Gap test of the state entering this iteration's prox step (one workgroup):
// eta = sum of the prox blocks' value and conjugate sums, checked from the
// second iteration on (the state after at least one projection).
template <typename T>
__device__ __forceinline__ void gap_check_body(const IterArgs<T> &p) {
  __shared__ double bs[kBlock / kWave];
  CtrlState &st = p.ctrl->st[p.par];
  if (st.done || st.k == 0) return;
  const int nb = p.nbx + p.nby;
  double o = 0.0, c = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) {
    o += p.s_gobj[i];
    c += p.s_gconj[i];
  }
  o = block_sum(o, bs);
  c = block_sum(c, bs);
  if (threadIdx.x == 0) {
    const double eta = o + c;
    const double eps = p.ctrl->eps_abs + p.ctrl->eps_rel * fabs(o);
    st.eta = eta;
    st.eps_gap = eps;
    if (eta < eps) {
      st.done = 1 + POGS_CONVERGED;
      st.by_gap = 1;
    }
  }
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

// Row epilogues gather a row's own inputs in pre(i) and finish it in
// row(i, s0, s1, pre) (row(i, s0, s1) is both in one call, the form every row
// pass uses).
template <typename T> struct Pre1 {
  T a;
};
template <typename T> struct Pre2 {
  T a, b;
};

// m >= n, solve: x = K^{-1} rhs
template <typename T> struct EpiTallSolve : EpiBase<T> {
  __device__ Pre1<T> pre(int j) const { return Pre1<T>{this->p.cx[j]}; }
  __device__ double row(int j, double x, double, const Pre1<T> &q) const {
    const IterArgs<T> &p = this->p;
    const T xv = (T)x;
    p.x[j] = xv;
    p.xt[j] = q.a - xv;
    return 0.0;
  }
  __device__ double row(int j, double x, double s) const { return row(j, x, s, pre(j)); }
  __device__ void block_done(int, double) const {}
};

// m >= n, pass 2: [y, t] = A [x, x_h]; then the stopping test
template <typename T> struct EpiTallPass2 : EpiBase<T> {
  __device__ Pre2<T> pre(int i) const { return Pre2<T>{this->p.dy[i], this->p.yh[i]}; }
  __device__ double row(int i, double y, double t, const Pre2<T> &q) const {
    const IterArgs<T> &p = this->p;
    const T yv = (T)y;
    p.y[i] = yv;
    p.yt[i] = q.a - yv;
    const double r = t - (double)q.b;
    return r * r;
  }
  __device__ double row(int i, double y, double t) const { return row(i, y, t, pre(i)); }
  __device__ void block_done(int b, double v) const { this->p.s_pri[b] = v; }
};

// m < n, pass 1: [u, t] = A [c, x_h]
template <typename T> struct EpiWidePass1 : EpiBase<T> {
  __device__ Pre2<T> pre(int i) const { return Pre2<T>{this->p.dy[i], this->p.yh[i]}; }
  __device__ double row(int i, double u, double t, const Pre2<T> &q) const {
    const IterArgs<T> &p = this->p;
    p.rhs[i] = (T)(u - (double)q.a);
    const double r = t - (double)q.b;
    return r * r;
  }
  __device__ double row(int i, double u, double t) const { return row(i, u, t, pre(i)); }
  __device__ void block_done(int b, double v) const { this->p.s_pri[b] = v; }
};

// m < n, solve: y = d + K^{-1} rhs, y~ = d - y
template <typename T> struct EpiWideSolve : EpiBase<T> {
  __device__ Pre1<T> pre(int i) const { return Pre1<T>{this->p.dy[i]}; }
  __device__ double row(int i, double z, double, const Pre1<T> &q) const {
    const IterArgs<T> &p = this->p;
    const T yv = (T)((double)q.a + z);
    p.y[i] = yv;
    p.yt[i] = q.a - yv;
    return 0.0;
  }
  __device__ double row(int i, double z, double s) const { return row(i, z, s, pre(i)); }
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

// ---------------------------------------------------------------------------
// Function parameters for the pre-conditioned problem (Section 4.1):
//   f^(y) = f(y / D):  a/D, b, c, d/D, e/D^2      (divide = true, scale = D)
//   g^(x) = g(E x):    a E, b, c, d E, e E^2      (divide = false, scale = E)
// Inputs are float64 per-element arrays; outputs in the iteration type.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void scale_fn_body(const Blk &blk, const uint8_t *h, const double *a, const double *b,
                                              const double *c, const double *d, const double *e,
                                              const double *scale, bool divide, int len, uint8_t *oh, T *oa, T *ob,
                                              T *oc, T *od, T *oe) {
  const int i = blk.x * kBlock + threadIdx.x;
  if (i >= len) return;
  const double s = scale ? (divide ? 1.0 / scale[i] : scale[i]) : 1.0;
  oh[i] = h[i];
  oa[i] = (T)(a[i] * s);
  ob[i] = (T)b[i];
  oc[i] = (T)c[i];
  od[i] = (T)(d[i] * s);
  oe[i] = (T)(e[i] * s * s);
}

// ---------------------------------------------------------------------------
// Return the half-step tuple in the original variables (Section 5):
//   x = E x_h, y = y_h / D, mu = mu_h / E, nu = D nu_h,
// and the objective f(y) + g(x) with the unscaled parameters.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void unscale_body(
    const Blk &b, const IterArgs<T> &p, const double *D, const double *E, const uint8_t *fh, const double *fa,
    const double *fb, const double *fc, const double *fd, const double *fe, const uint8_t *gh,
    const double *ga, const double *gb, const double *gc, const double *gd, const double *ge, T *xo,
    T *yo, T *muo, T *nuo, double *slots, double *obj, unsigned *cnt, int from_state = 0, double rho = 0.0) {
  __shared__ double bs[kBlock / kWave];
  __shared__ int flag;
  const bool xs = b.x < p.nbx;
  const int blk = xs ? b.x : b.x - p.nbx;
  const int i = blk * kBlock + threadIdx.x;
  double contrib = 0.0;
  if (xs && i < p.n) {
    const double xv = from_state ? (double)p.x[i] : (double)p.xh[i];
    const double mv = from_state ? -rho * (double)p.xt[i] : (double)p.mu[i];
    const double x = E[i] * xv;
    if (xo) xo[i] = (T)x;
    if (muo) muo[i] = (T)(mv / E[i]);
    contrib = fn_value(gh[i], ga[i], gb[i], gc[i], gd[i], ge[i], x);
  } else if (!xs && i < p.m) {
    const double yv = from_state ? (double)p.y[i] : (double)p.yh[i];
    const double nv = from_state ? -rho * (double)p.yt[i] : (double)p.nu[i];
    const double y = yv / D[i];
    if (yo) yo[i] = (T)y;
    if (nuo) nuo[i] = (T)(D[i] * nv);
    contrib = fn_value(fh[i], fa[i], fb[i], fc[i], fd[i], fe[i], y);
  }
  const double s = block_sum(contrib, bs);
  if (threadIdx.x == 0) slots[b.x] = s;
  if (arrive_last(cnt, b.nx, &flag)) {
    double t = 0.0;
    for (int j = threadIdx.x; j < b.nx; j += blockDim.x) t += load_agent(slots + j);
    const double tot = block_sum(t, bs);
    if (threadIdx.x == 0) *obj = tot;
  }
}

// out = f * (v0 / S) or f * (v0 * S), elementwise (the warm start's change of variables)
template <typename T>
__global__ __launch_bounds__(kBlock) void warm_scale_kernel(const T *v0, const double *S, bool divide, double f,
                                                            int len, T *out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < len) out[i] = (T)(f * (divide ? (double)v0[i] / S[i] : (double)v0[i] * S[i]));
}

}  // namespace pogs
