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
// This thread's sum of slots threadIdx.x, threadIdx.x + blockDim.x, ... of s
// (in that order).  The first kSlotUnroll loads are issued together: a loop
// whose trip count the compiler cannot see waits for each load before the
// next, and these slot loads open every kernel that runs the stop test.
// The sums are taken over kBlock threads whatever the workgroup size, so that
// a wider workgroup (with its other threads adding zeros) gets the same bits.
constexpr int kSlotUnroll = 4;
__device__ inline double slot_partial(const double *s, int cnt) {
  if ((int)threadIdx.x >= kBlock) return 0.0;
  double v[kSlotUnroll];
#pragma unroll
  for (int k = 0; k < kSlotUnroll; ++k) {
    const int i = threadIdx.x + k * kBlock;
    v[k] = i < cnt ? s[i] : 0.0;
  }
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < kSlotUnroll; ++k) t += v[k];
  for (int i = threadIdx.x + kSlotUnroll * kBlock; i < cnt; i += kBlock) t += s[i];
  return t;
}

template <typename T>
__device__ inline void control_partials(const IterArgs<T> &p, int spar, double part[4]) {
  part[0] = slot_partial(p.s_mu + (size_t)spar * p.n_smu, p.n_smu);
  part[1] = slot_partial(p.s_yh + (size_t)spar * p.n_syh, p.n_syh);
  part[2] = slot_partial(p.s_pri, p.n_pri);
  part[3] = slot_partial(p.s_dual, p.n_dual);
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


// One element of the prox step (Algorithm 1 with over-relaxation, Section
// 3.2, and the half-step dual of Section 3.3): the pending rescale of the
// scaled dual vt, the half step h = prox(v - vt), its dual -rho (h - (v - vt))
// and the projection input alpha h + (1 - alpha) v + vt.
template <typename T> struct HalfStep {
  T h, dual, proj_in, vt;
};
template <typename T>
__device__ __forceinline__ HalfStep<T> half_step(int fh, T fa, T fb, T fc, T fd, T fe, T v, T vt, T rho, T resc,
                                                 T alpha) {
  HalfStep<T> r;
  if (resc != T(1)) vt *= resc;
  const T arg = v - vt;
  r.h = prox_param<T>(fh, fa, fb, fc, fd, fe, arg, rho);
  r.dual = -rho * (r.h - arg);
  const T rel = alpha * r.h + (T(1) - alpha) * v;
  r.proj_in = rel + vt;
  r.vt = vt;
  return r;
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
    const HalfStep<T> hs = half_step<T>(fh, fa, fb, fc, fd, fe, vi, vti, rho, resc, alpha);
    if constexpr (!CG) {
      if (resc != T(1)) vt[i] = hs.vt;
    }
    if (gap) {
      // the state is primal and dual feasible: value at (x, y), conjugate at
      // (mu, nu) = (-rho x~, -rho y~)
      gobj = fn_value_strict(fh, fa, fb, fc, fd, fe, (double)vi);
      gconj = fn_conj_value(fh, fa, fb, fc, fd, fe, -(double)st.rho * (double)hs.vt);
    }
    const T h = hs.h, dual = hs.dual;
    if (xs) {
      p.xh[i] = h;
      p.mu[i] = dual;
      p.cx[i] = hs.proj_in;
      if constexpr (CG) p.x[i] = h;
    } else {
      p.yh[i] = h;
      p.nu[i] = dual;
      p.dy[i] = hs.proj_in;
    }
    contrib = xs ? (double)dual * (double)dual : (double)h * (double)h;
  }
  const double s = block_sum(contrib, bs);
  if (threadIdx.x == 0) {
    if (xs) p.s_mu[(size_t)par * p.n_smu + blk] = s;
    else p.s_yh[(size_t)par * p.n_syh + blk] = s;
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

// ---------------------------------------------------------------------------
// Fused tall iteration (m >= n, direct projection, residual stopping): the
// prox step runs inside the first pass and its finish, so an iteration is
// four launches (pass 1, its finish, the solve, pass 2) instead of five.
//   pass 1, workgroup (tile, split): the stop test and Algorithm 3 of the
//     previous iteration (as in prox_body), then for the split's rows the y
//     side of the prox step (every column tile computes it for its own use;
//     tile 0 stores y_h, nu_h, d and sums ||y_h||^2 per split), then the
//     split partials of [w, s] = A^T [d, nu_h];
//   finish, kFinishCols columns per workgroup: the x side of the prox step
//     per column (x_h, mu_h, c), rhs = c + w, and per tile the sums of
//     (s + mu_h)^2 and mu_h^2.
// The rescale of (x~, y~) is applied where the values are read and not
// stored back: the solve and pass 2 overwrite x~ and y~ in this iteration.
// The column sums follow gemv_t_body's per-lane order exactly.
// ---------------------------------------------------------------------------
constexpr int kProxRows = 1024;  // rows of one split whose (d, nu_h) sit in LDS at a time
constexpr int kProxRowsPerThread = kProxRows / kBlock;

// In the one-pass iteration this kernel mostly runs only the stop test (the
// previous iteration's results stand), so nothing else is loaded before it.
// When it does run the pass, groups of 8 rows are loaded and used one at a
// time (measured on gfx950 at 20000 x 2000: 24.5 us against 26.9 us with two
// groups in flight).
template <typename T, bool NT>
__device__ __forceinline__ void tall_pass1_prox_body(const Blk &b, const IterArgs<T> &p, int rows_per_split,
                                                     int ncolp) {
  using V = typename Vec16<T>::type;
  constexpr int VN = Vec16<T>::N;
  constexpr int TILE = kWave * VN;
  constexpr int PR = kProxRowsPerThread;
  __shared__ double red[4][2][TILE];
  __shared__ T dv[kProxRows], nv[kProxRows];
  __shared__ double bs[4 * (kBlock / kWave)];
  __shared__ CtrlState st;
  const int par = p.par;
  const int tile = b.x, split = b.y;
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int col = tile * TILE + lane * VN;
  const int r0 = split * rows_per_split;
  const int r1 = min(p.m, r0 + rows_per_split);
  const int ld = p.ld;
  const bool colok = col < p.n;
  const T *base = p.A + (colok ? col : 0);
  auto group_load = [&](V *dst, int i) {
#pragma unroll
    for (int u = 0; u < 8; ++u) dst[u] = mat_load<NT>(reinterpret_cast<const V *>(base + (size_t)(i + 4 * u) * ld));
  };
  // prox inputs of the rows c0 + threadIdx.x + k kBlock of a chunk
  T py[PR], pyt[PR], pa[PR], pb[PR], pc[PR], pd[PR], pe[PR];
  int ph[PR];
  auto prox_load = [&](int c0, int c1) {
#pragma unroll
    for (int k = 0; k < PR; ++k) {
      const int i = c0 + threadIdx.x + k * kBlock;
      if (i < c1) {
        py[k] = p.y[i];
        pyt[k] = p.yt[i];
        ph[k] = p.f.h[i];
        pa[k] = p.f.a[i];
        pb[k] = p.f.b[i];
        pc[k] = p.f.c[i];
        pd[k] = p.f.d[i];
        pe[k] = p.f.e[i];
      }
    }
  };

  __shared__ double spec_rho;
  if (threadIdx.x == 0) {
    st = p.ctrl->st[1 - par];
    spec_rho = p.ctrl->spec_rho[par];
  }
  double part[4];
  control_partials(p, 1 - par, part);
  V a[8];
  __syncthreads();
  const bool after_iteration = st.pending != 0;  // an iteration ran before this one in the solve
  if (!st.done && st.pending) control_apply(p, part, st, bs);
  // the previous iteration's one-pass kernel computed this step with the rho
  // Algorithm 3 has just chosen (and the matching rescale): its results stand
  const bool spec = after_iteration && !st.done && st.rho == spec_rho;
  if (b.x == 0 && b.y == 0 && threadIdx.x == 0) {
    CtrlState out = st;
    out.pending = st.done ? 0 : 1;
    out.spec = spec ? 1 : 0;
    p.ctrl->st[par] = out;
  }
  if (st.done || spec) return;
  if (b.x == 0 && b.y == 0)  // the slots of ||y_h||^2 past this launch's splits
    for (int j = b.ny + threadIdx.x; j < p.n_syh; j += kBlock) p.s_yh[(size_t)par * p.n_syh + j] = 0.0;
  const int c1_first = min(r1, r0 + kProxRows);
  const bool pre = colok && r0 + w + 28 < c1_first;
  if (pre) group_load(a, r0 + w);
  prox_load(r0, c1_first);
  const T rho = (T)st.rho, resc = (T)st.rescale, alpha = (T)p.ctrl->alpha;
  const bool store = tile == 0;

  double acc[2][VN];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < VN; ++c) acc[r][c] = 0.0;
  auto group_fma = [&](int i, int c0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double s0 = (double)dv[i + 4 * u - c0], s1 = (double)nv[i + 4 * u - c0];
#pragma unroll
      for (int c = 0; c < VN; ++c) {
        const double e = (double)a[u][c];
        acc[0][c] = fma(e, s0, acc[0][c]);
        acc[1][c] = fma(e, s1, acc[1][c]);
      }
    }
  };

  double yh2 = 0.0;
  for (int c0 = r0; c0 < r1; c0 += kProxRows) {
    const int c1 = min(r1, c0 + kProxRows);
    if (c0 != r0) prox_load(c0, c1);
    // y side of the prox step for rows c0 .. c1 - 1
#pragma unroll
    for (int k = 0; k < PR; ++k) {
      const int i = c0 + threadIdx.x + k * kBlock;
      if (i < c1) {
        const HalfStep<T> hs = half_step<T>(ph[k], pa[k], pb[k], pc[k], pd[k], pe[k], py[k], pyt[k], rho, resc, alpha);
        dv[i - c0] = hs.proj_in;
        nv[i - c0] = hs.dual;
        if (store) {
          p.yh[i] = hs.h;
          p.nu[i] = hs.dual;
          p.dy[i] = hs.proj_in;
          yh2 += (double)hs.h * (double)hs.h;
        }
      }
    }
    __syncthreads();
    if (colok) {
      int i = c0 + w;
      if (i + 28 < c1) {  // the first group was loaded before the stop test in the first chunk
        if (c0 != r0 || !pre) group_load(a, i);
        group_fma(i, c0);
        i += 32;
      }
      for (; i + 28 < c1; i += 32) {
        group_load(a, i);
        group_fma(i, c0);
      }
      for (; i < c1; i += 4) {
        const V x = mat_load<NT>(reinterpret_cast<const V *>(base + (size_t)i * ld));
        const double s0 = (double)dv[i - c0], s1 = (double)nv[i - c0];
#pragma unroll
        for (int c = 0; c < VN; ++c) {
          const double e = (double)x[c];
          acc[0][c] = fma(e, s0, acc[0][c]);
          acc[1][c] = fma(e, s1, acc[1][c]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int c = 0; c < VN; ++c) red[w][r][lane * VN + c] = acc[r][c];
  __syncthreads();
  if (threadIdx.x < TILE) {
    const int t = threadIdx.x;
    const int cg = tile * TILE + t;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const double v = (red[0][r][t] + red[1][r][t]) + (red[2][r][t] + red[3][r][t]);
      p.part[(size_t)(split * 2 + r) * ncolp + cg] = v;
    }
  }
  if (store) {
    const double s = block_sum(yh2, bs);
    if (threadIdx.x == 0) p.s_yh[(size_t)par * p.n_syh + split] = s;
  }
}

// Finish of the first pass of the tall iteration: split sums of kFinishCols
// columns (in the order of gemv_t_finish_body), then per column the x side of
// the prox step, rhs = c + w and the tile sums of (s + mu_h)^2 and mu_h^2.
// The splits are the one-pass kernel's workgroups when its results stand,
// else the first pass's row splits.  The column's own inputs and up to
// kFinishLoads split partials per thread are loaded together.
constexpr int kFinishLoads = 32;
template <typename T>
__device__ __forceinline__ void tall_finish_prox_body(const Blk &b, const IterArgs<T> &p, int splits, int ncolp) {
  constexpr int G = kBlock / kFinishCols;
  __shared__ double red[G][2][kFinishCols];
  __shared__ double bs[kBlock / kWave];
  const CtrlState &gst = p.ctrl->st[p.par];  // stored by the first pass's workgroup (0, 0)
  const int c = threadIdx.x % kFinishCols;
  const int g = threadIdx.x / kFinishCols;
  const int cg = b.x * kFinishCols + c;
  const bool mine = g == 0 && cg < p.n;
  T xv = T(0), xtv = T(0), fa = T(0), fb = T(0), fc = T(0), fd = T(0), fe = T(0);
  int fh = 0;
  if (mine) {
    xv = p.x[cg];
    xtv = p.xt[cg];
    fh = p.g.h[cg];
    fa = p.g.a[cg];
    fb = p.g.b[cg];
    fc = p.g.c[cg];
    fd = p.g.d[cg];
    fe = p.g.e[cg];
  }
  const int nsp = gst.spec ? p.fp_blocks : splits;
  double s[2] = {0.0, 0.0};
  if (cg < ncolp) {
    double v0[kFinishLoads], v1[kFinishLoads];
#pragma unroll
    for (int k = 0; k < kFinishLoads; ++k) {
      const int sp = g + k * G;
      v0[k] = sp < nsp ? p.part[(size_t)(sp * 2) * ncolp + cg] : 0.0;
      v1[k] = sp < nsp ? p.part[(size_t)(sp * 2 + 1) * ncolp + cg] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < kFinishLoads; ++k) {
      s[0] += v0[k];
      s[1] += v1[k];
    }
    for (int sp = g + kFinishLoads * G; sp < nsp; sp += G) {
      s[0] += p.part[(size_t)(sp * 2) * ncolp + cg];
      s[1] += p.part[(size_t)(sp * 2 + 1) * ncolp + cg];
    }
  }
  if (gst.done) return;  // checked after the loads were issued (reading is harmless once stopped)
  red[g][0][c] = s[0];
  red[g][1][c] = s[1];
  __syncthreads();
  double dual2 = 0.0, mu2 = 0.0;
  if (mine) {
    double t0 = 0.0, t1 = 0.0;
#pragma unroll
    for (int k = 0; k < G; ++k) {
      t0 += red[k][0][c];
      t1 += red[k][1][c];
    }
    const HalfStep<T> hs = half_step<T>(fh, fa, fb, fc, fd, fe, xv, xtv, (T)gst.rho, (T)gst.rescale,
                                        (T)p.ctrl->alpha);
    p.xh[cg] = hs.h;
    p.mu[cg] = hs.dual;
    p.cx[cg] = hs.proj_in;
    p.rhs[cg] = (T)((double)hs.proj_in + t0);
    const double r = t1 + (double)hs.dual;
    dual2 = r * r;
    mu2 = (double)hs.dual * (double)hs.dual;
  }
  const double ta = block_sum(dual2, bs);
  const double tb = block_sum(mu2, bs);
  if (threadIdx.x == 0) {
    p.s_dual[b.x] = ta;
    p.s_mu[(size_t)p.par * p.n_smu + b.x] = tb;
  }
}

// ---------------------------------------------------------------------------
// One pass over A per tall iteration (float32 A, rows of at most 256 NC
// entries).  While a row of A is in registers the kernel finishes iteration k
// (second pass: y = A x, t = A x_h, y~ = d - y, (t - y_h)^2) and starts
// iteration k + 1: the y side of its prox step from the y, y~ just formed,
// then that row's share of the column sums A^T [d', nu_h'].  The half step
// needs the rho that Algorithm 3 picks after iteration k.  Of its inputs only
// the primal residual is still open here (the dual residual and both
// tolerances are final once the first pass's finish has run), so each
// workgroup evaluates the rule with those values and takes, for the open
// test, the outcome of the previous iteration's.  When the stop test after
// iteration k picks another rho (or stops), the next first-pass kernel
// recomputes those values (tall_pass1_prox_body) and these are discarded.
// Iteration k + 1's half step goes to the other half-step set, so iteration
// k's (the result, should the stop test end the solve here) stays.
// Workgroups of kOnePassThreads; wave gw takes a contiguous run of rows (the
// first m mod W waves one row more than the others), so the inputs and
// outputs of a batch of its rows are contiguous.  Lane l keeps the column
// sums of columns 4 l + 256 u + c (u < NC, c < 4) over its rows, in float64
// for rows of at most 1024 entries and in float32 for longer rows (64 float64
// sums per lane would not fit the registers of two waves per SIMD;
// one_pass_blocks keeps those waves at 64 rows or fewer); the waves' sums are
// added in LDS in float64 in wave order and each workgroup writes one split
// partial.  Every lane finishes each row (the row's sums are the same in all
// lanes after wave_sum), so no value has to be broadcast.
// ---------------------------------------------------------------------------
constexpr int kOnePassThreads = 512;
template <int NC, bool NT>
__device__ __forceinline__ void tall_one_pass_body(const Blk &b, const IterArgs<float> &p, int ncolp) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int NW = kOnePassThreads / kWave;
  constexpr int CH = 64 * NC;                                   // 16-byte pieces of a staged vector
  constexpr int CPT = (CH + kOnePassThreads - 1) / kOnePassThreads;
  using Acc = typename std::conditional<(NC >= 8), float, double>::type;
  __shared__ float xs[2][256 * NC];
  __shared__ Acc red[NW][2][256 * NC];  // every wave's column sums (128 KB)
  __shared__ double bs[4 * NW];
  __shared__ double rho_next;
  const CtrlState &gst = p.ctrl->st[p.par];
  const bool stopped = gst.done != 0;  // used once the first loads are out
  // every control value the rho rule reads, loaded with the first loads (read
  // after the barriers below they would cost another round trip to memory)
  const Ctrl &q = *p.ctrl;
  const double st_rho = gst.rho, st_rpri = gst.r_pri, st_epri = gst.eps_pri;
  const int st_k = gst.k, st_l = gst.l, st_u = gst.u;
  const double q_eabs = q.eps_abs, q_erel = q.eps_rel, q_tau = q.tau, q_delta = q.delta;
  const float alpha = (float)q.alpha;
  const int q_adaptive = q.adaptive;
  double part[4];
  part[0] = slot_partial(p.s_mu + (size_t)p.par * p.n_smu, p.n_smu);
  part[1] = part[2] = 0.0;  // the primal tolerance is not needed (see below)
  part[3] = slot_partial(p.s_dual, p.n_dual);
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x >> 6;
  const int W = b.nx * NW;
  const int gw = __builtin_amdgcn_readfirstlane(b.x * NW + w);
  const int m = p.m, n = p.n, ld = p.ld;
  const float *A = p.A;

  // x (this iteration's projection) and x_h (its half step): context vectors, 16-byte aligned
  f4 stg[2][CPT];
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int q = threadIdx.x + kOnePassThreads * j;
    const int idx = 4 * q;
    if (q < CH) {
      if (idx + 3 < n) {
        stg[0][j] = *reinterpret_cast<const f4 *>(p.x + idx);
        stg[1][j] = *reinterpret_cast<const f4 *>(p.xh + idx);
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          stg[0][j][k] = idx + k < n ? p.x[idx + k] : 0.f;
          stg[1][j][k] = idx + k < n ? p.xh[idx + k] : 0.f;
        }
      }
    }
  }
  const int rq = m / W, rr = m % W;
  const int nrows = rq + (gw < rr ? 1 : 0);
  const int row0 = gw * rq + min(gw, rr);
  int cofs[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) cofs[u] = min(4 * lane + 256 * u, ld - 4);
  auto load = [&](f4 *dst, int r) {
    const float *rp = A + (size_t)r * ld;
#pragma unroll
    for (int u = 0; u < NC; ++u) dst[u] = mat_load<NT>(reinterpret_cast<const f4 *>(rp + cofs[u]));
  };
  f4 a0[NC], a1[NC];
  if (nrows > 0) load(a0, row0);
  // Rows go in batches of up to 64: lane t loads the inputs of the batch's row
  // t up front and keeps its outputs until the batch ends, so the row loop
  // itself issues no memory access other than the rows of A (a load or store
  // between two rows makes the compiler wait for everything in flight).  Row
  // t's inputs reach every lane by readlane.  The first batch's inputs are
  // loaded here, with the first row.
  float b_dy = 0.f, b_yh = 0.f, b_fa = 0.f, b_fb = 0.f, b_fc = 0.f, b_fd = 0.f, b_fe = 0.f;
  int b_fh = 0;
  auto load_inputs = [&](int i0) {
    if (lane < min(kWave, nrows - i0)) {
      const int mine = row0 + i0 + lane;
      b_dy = p.dy[mine];
      b_yh = p.yh[mine];
      b_fh = p.f.h[mine];
      b_fa = p.f.a[mine];
      b_fb = p.f.b[mine];
      b_fc = p.f.c[mine];
      b_fd = p.f.d[mine];
      b_fe = p.f.e[mine];
    }
  };
  load_inputs(0);
  if (stopped) return;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    const int q = threadIdx.x + kOnePassThreads * j;
    if (q < CH) {
      *reinterpret_cast<f4 *>(&xs[0][4 * q]) = stg[0][j];
      *reinterpret_cast<f4 *>(&xs[1][4 * q]) = stg[1][j];
    }
  }
  // the sums are those of control_apply bit for bit (threads past kBlock add zeros)
  block_sum4(part, bs);
  if (threadIdx.x == 0) {
    const double r_dual = sqrt(part[3]);
    const double eps_dual = q_eabs + q_erel * sqrt(part[0]);
    double next = st_rho;
    if (q_adaptive) {
      if (r_dual < eps_dual && q_tau * st_k > st_l) next = q_delta * st_rho;
      else if (st_rpri < st_epri && q_tau * st_k > st_u) next = st_rho / q_delta;
    }
    rho_next = next;
    if (b.x == 0) p.ctrl->spec_rho[1 - p.par] = next;
  }
  __syncthreads();
  const double rho_d = rho_next;
  const float rho = (float)rho_d, resc = (float)(rho_d != st_rho ? st_rho / rho_d : 1.0);

  Acc acc[2][NC][4];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int u = 0; u < NC; ++u)
#pragma unroll
      for (int k = 0; k < 4; ++k) acc[r][u][k] = Acc(0);
  double pri = 0.0, yh2 = 0.0;
  float o_y = 0.f, o_yt = 0.f, o_h = 0.f, o_nu = 0.f, o_d = 0.f;
  auto bcast = [](float v, int t) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), t)); };
  auto row = [&](const f4 *a, int t) {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      const f4 x0 = *reinterpret_cast<const f4 *>(&xs[0][4 * lane + 256 * u]);
      const f4 x1 = *reinterpret_cast<const f4 *>(&xs[1][4 * lane + 256 * u]);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double e = (double)a[u][k];
        s0 = fma(e, (double)x0[k], s0);
        s1 = fma(e, (double)x1[k], s1);
      }
      // widest rows: keep the scheduler from hoisting every LDS read and
      // conversion of the row at once (that spills)
      if constexpr (NC >= 8) __builtin_amdgcn_sched_barrier(0);
    }
    s0 = wave_sum_dpp(s0);
    s1 = wave_sum_dpp(s1);
    // iteration k: y = A x, y~ = d - y, (A x_h - y_h)^2
    const float yv = (float)s0;
    const float ytv = bcast(b_dy, t) - yv;
    const double r = s1 - (double)bcast(b_yh, t);
    pri += r * r;
    // iteration k + 1: y side of the half step with the predicted rho
    const HalfStep<float> hs = half_step<float>(__builtin_amdgcn_readlane(b_fh, t), bcast(b_fa, t), bcast(b_fb, t),
                                                bcast(b_fc, t), bcast(b_fd, t), bcast(b_fe, t), yv, ytv, rho, resc,
                                                alpha);
    yh2 += (double)hs.h * (double)hs.h;
    if (lane == t) {
      o_y = yv;
      o_yt = ytv;
      o_h = hs.h;
      o_nu = hs.dual;
      o_d = hs.proj_in;
    }
    const Acc d0 = (Acc)hs.proj_in, d1 = (Acc)hs.dual;
#pragma unroll
    for (int u = 0; u < NC; ++u)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const Acc e = (Acc)a[u][k];
        acc[0][u][k] = fma(e, d0, acc[0][u][k]);
        acc[1][u][k] = fma(e, d1, acc[1][u][k]);
      }
  };
  // row i of the wave is in a0 for even i and a1 for odd i (batches are 64 rows)
  for (int i0 = 0; i0 < nrows; i0 += kWave) {
    const int cnt = min(kWave, nrows - i0);
    const int mine = row0 + i0 + lane;
    if (i0 > 0) load_inputs(i0);
    for (int t = 0; t < cnt; t += 2) {
      const int i = i0 + t;
      if (i + 1 < nrows) load(a1, row0 + i + 1);
      row(a0, t);
      if (t + 1 >= cnt) break;
      if (i + 2 < nrows) load(a0, row0 + i + 2);
      row(a1, t + 1);
    }
    if (lane < cnt) {
      p.y[mine] = o_y;
      p.yt[mine] = o_yt;
      p.nyh[mine] = o_h;
      p.nnu[mine] = o_nu;
      p.ndy[mine] = o_d;
    }
  }
  // the workgroup's column sums: the waves' sums added in float64 in wave order
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int u = 0; u < NC; ++u)
#pragma unroll
      for (int k = 0; k < 4; ++k) red[w][r][4 * lane + 256 * u + k] = acc[r][u][k];
  if (lane == 0) {  // pri and yh2 are the same in every lane of the wave
    bs[w] = pri;
    bs[NW + w] = yh2;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < ncolp; j += kOnePassThreads) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < NW; ++q) v += (double)red[q][r][j];
      p.part[(size_t)(b.x * 2 + r) * ncolp + j] = v;
    }
  }
  if (threadIdx.x == 0) {  // the waves in index order (the bits of block_sum)
    double sp = 0.0, sy = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
      sp += bs[k];
      sy += bs[NW + k];
    }
    p.s_pri[b.x] = sp;
    p.s_yh[(size_t)(1 - p.par) * p.n_syh + b.x] = sy;
  }
  if (b.x == 0)  // the slots of ||y_h'||^2 past this launch's workgroups
    for (int j = b.nx + threadIdx.x; j < p.n_syh; j += kOnePassThreads) p.s_yh[(size_t)(1 - p.par) * p.n_syh + j] = 0.0;
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

// The half of a warm start the caller left out (Section 5: it is
// estimated), as one proximal point step from zero, the value the prox step
// of the iteration returns: primal = 0 -> out = prox_F(v) - v (the scaled
// dual y~ from y; nu^ = rho (y - prox_f^(y))); primal = 1 -> out = prox_F(-v)
// (x from the scaled dual x~: prox_g^(mu^ / rho) with mu^ = -A^T nu^ = -rho x~).
template <typename T>
__global__ __launch_bounds__(kBlock) void warm_estimate_kernel(FnDev<T> F, const T *v, T *out, int len, T rho,
                                                               int primal) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= len) return;
  const T vi = v[i];
  if (primal) out[i] = prox_param<T>(F.h[i], F.a[i], F.b[i], F.c[i], F.d[i], F.e[i], -vi, rho);
  else out[i] = prox_param<T>(F.h[i], F.a[i], F.b[i], F.c[i], F.d[i], F.e[i], vi, rho) - vi;
}

// out = f * (v0 / S) or f * (v0 * S), elementwise (the warm start's change of variables)
template <typename T>
__global__ __launch_bounds__(kBlock) void warm_scale_kernel(const T *v0, const double *S, bool divide, double f,
                                                            int len, T *out) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < len) out[i] = (T)(f * (divide ? (double)v0[i] / S[i] : (double)v0[i] * S[i]));
}

}  // namespace pogs
