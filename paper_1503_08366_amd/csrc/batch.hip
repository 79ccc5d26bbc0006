// Persistent batched solver: each 256-thread workgroup takes a problem from
// the device work queue and runs, inside the workgroup,
//   setup      : Algorithm 2 sweeps + Frobenius normalisation (Sections 4.1.2,
//                4.2, 5), A <- D A E, pre-conditioned function parameters,
//                Gram matrix on f32 MFMA, blocked float64 Cholesky of I + G,
//                blocked L^{-1} and K^{-1} = L^{-T} L^{-1} on f64 MFMA;
//   iterations : Algorithm 1 with relaxation (Section 3.2), half-step duals
//                (Section 3.3), residual stopping (Section 3.4) and Algorithm 3,
//                the same steps as the whole-GPU pipeline but with
//                workgroup-level passes over A;
//   finish     : the half-step tuple in the original variables and f(y) + g(x).
// A problem's arithmetic does not depend on which workgroup runs it, on the
// other problems, or on how its iterations are split over launches (its state
// lives in device memory between launches), so a problem gives the same bits
// alone or in any mix.
#include "batch.hpp"
#include "factor.hpp"
#include "prox.hpp"

namespace pogs {

namespace {

constexpr int kThreads = 256;

typedef double RedBuf[4][2][256];  // gemv_t cross-wave reduction (in the dynamic LDS)

struct WgShared {
  double bs[kThreads / kWave];
  int idx;
  int done;
  float rho, rescale;
};

// Column sums over A (m x n, leading dim ld): s_r[j] = sum_i op(A_ij) v_r[i];
// column(j, s0, s1) finishes column j and returns a value summed over j (the
// block total is returned in thread 0).
template <bool SQUARE, int NRHS, typename TV, class Col>
__device__ double wg_gemv_t(const float *__restrict__ A, int m, int n, int ld, const TV *v0, const TV *v1,
                            char *lds, WgShared &sh, Col column) {
  RedBuf &red = *reinterpret_cast<RedBuf *>(lds);
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  double contrib = 0.0;
  typedef float f4 __attribute__((ext_vector_type(4)));
  for (int ct = 0; ct < n; ct += 256) {
    const int col = ct + lane * 4;
    double acc[NRHS][4];
#pragma unroll
    for (int r = 0; r < NRHS; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
    if (col < n) {
      const float *base = A + col;
      int i = w;
      for (; i + 28 < m; i += 32) {
        f4 a[8];
        double s[8][NRHS];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          a[u] = *reinterpret_cast<const f4 *>(base + (size_t)(i + 4 * u) * ld);
          s[u][0] = (double)v0[i + 4 * u];
          if constexpr (NRHS > 1) s[u][1] = (double)v1[i + 4 * u];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            double e = (double)a[u][c];
            if constexpr (SQUARE) e *= e;
#pragma unroll
            for (int r = 0; r < NRHS; ++r) acc[r][c] = fma(e, s[u][r], acc[r][c]);
          }
      }
      for (; i < m; i += 4) {
        const f4 a = *reinterpret_cast<const f4 *>(base + (size_t)i * ld);
        double s[NRHS];
        s[0] = (double)v0[i];
        if constexpr (NRHS > 1) s[1] = (double)v1[i];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          double e = (double)a[c];
          if constexpr (SQUARE) e *= e;
#pragma unroll
          for (int r = 0; r < NRHS; ++r) acc[r][c] = fma(e, s[r], acc[r][c]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NRHS; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) red[w][r][lane * 4 + c] = acc[r][c];
    __syncthreads();
    {
      const int t = threadIdx.x;
      const int cg = ct + t;
      if (cg < n) {
        const double s0 = (red[0][0][t] + red[1][0][t]) + (red[2][0][t] + red[3][0][t]);
        double s1 = 0.0;
        if constexpr (NRHS > 1) s1 = (red[0][1][t] + red[1][1][t]) + (red[2][1][t] + red[3][1][t]);
        contrib += column(cg, s0, s1);
      }
    }
    __syncthreads();
  }
  return block_sum(contrib, sh.bs);
}

// Row dots over A (m x ncols, leading dim ld): s_r[i] = sum_j op(A_ij) v_r[j],
// the vectors staged in LDS (`vs`, 2 x ldv elements of TV).  LPR lanes per row
// chosen so each lane issues about 8 vector loads per row.
template <bool SQUARE, int NRHS, typename TV, class Row>
__device__ double wg_gemv_n(const float *__restrict__ A, int m, int ncols, int ld, const TV *v0, const TV *v1,
                            TV *vs, WgShared &sh, Row row) {
  const int ldv = (ncols + 63) & ~63;  // <= ld
  for (int t = threadIdx.x; t < ldv; t += kThreads) {
    vs[t] = t < ncols ? v0[t] : TV(0);
    if constexpr (NRHS > 1) vs[ldv + t] = t < ncols ? v1[t] : TV(0);
  }
  __syncthreads();
  const int nv = ldv / 4;
  int lpr = 4;
  while (lpr < 64 && lpr * 8 < nv) lpr *= 2;
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int sub = lane & (lpr - 1);
  const int gpw = 64 / lpr;
  const int grp = lane / lpr;
  typedef float f4 __attribute__((ext_vector_type(4)));
  double contrib = 0.0;
  for (int r0 = w * gpw + grp; r0 - grp < m; r0 += 4 * gpw) {
    double a0 = 0.0, a1 = 0.0;
    if (r0 < m) {
      const float *rowp = A + (size_t)r0 * ld;
#pragma unroll 4
      for (int c = sub * 4; c < ldv; c += lpr * 4) {
        const f4 a = *reinterpret_cast<const f4 *>(rowp + c);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          double e = (double)a[k];
          if constexpr (SQUARE) e *= e;
          a0 = fma(e, (double)vs[c + k], a0);
          if constexpr (NRHS > 1) a1 = fma(e, (double)vs[ldv + c + k], a1);
        }
      }
    }
    for (int o = lpr / 2; o > 0; o >>= 1) {
      a0 += __shfl_xor(a0, o, 64);
      if constexpr (NRHS > 1) a1 += __shfl_xor(a1, o, 64);
    }
    if (sub == 0 && r0 < m) contrib += row(r0, a0, a1);
  }
  const double tot = block_sum(contrib, sh.bs);
  __syncthreads();  // vs may be restaged by the next call
  return tot;
}

// --------------------------------------------------------------------------
// setup of one problem
// --------------------------------------------------------------------------
__device__ void wg_setup(BProb &P, double *ws, char *lds, WgShared &sh) {
  const int m = P.m, n = P.n, ld = P.ld, q = P.q, Q = P.Q;
  const int t = threadIdx.x;
  float *A = P.A;
  // non-finite entries
  unsigned nbad = 0;
  for (int i = 0; i < m; ++i)
    for (int j = t; j < n; j += kThreads)
      if (!isfinite(A[(size_t)i * ld + j])) ++nbad;
  if (nbad) atomicAdd(&P.bad, nbad);
  // ---- equilibration (Algorithm 2, p = 2) ----
  double *d = P.D, *e = P.E;
  if (P.equil_iters > 0) {
    const double gm = P.gamma / m, gn = P.gamma / n;
    for (int j = t; j < n; j += kThreads) e[j] = 1.0;
    __syncthreads();
    double fro2 = 0.0;
    for (int it = 0; it < P.equil_iters; ++it) {
      wg_gemv_n<true, 1, double>(A, m, n, ld, e, e, (double *)lds, sh, [&](int i, double s, double) {
        d[i] = (double)n / (s + gm);
        return 0.0;
      });
      __syncthreads();
      fro2 = wg_gemv_t<true, 1, double>(A, m, n, ld, d, d, lds, sh, [&](int j, double s, double) {
        const double ej = (double)m / (s + gn);
        e[j] = ej;
        return ej * s;
      });
      __syncthreads();
    }
    if (t == 0) sh.bs[0] = sqrt(fro2 / (double)q);
    __syncthreads();
    const double s = sh.bs[0];
    __syncthreads();
    for (int i = t; i < m; i += kThreads) d[i] = sqrt(d[i] / s);
    for (int j = t; j < n; j += kThreads) e[j] = sqrt(e[j] / s);
    __syncthreads();
    for (int i = 0; i < m; ++i)
      for (int j = t; j < n; j += kThreads) A[(size_t)i * ld + j] = (float)(d[i] * (double)A[(size_t)i * ld + j] * e[j]);
  } else {
    for (int i = t; i < m; i += kThreads) d[i] = 1.0;
    for (int j = t; j < n; j += kThreads) e[j] = 1.0;
  }
  // ---- pre-conditioned functions: f^(y) = f(y / D), g^(x) = g(E x) ----
  for (int i = t; i < m; i += kThreads) {
    const double s = 1.0 / d[i];
    P.fs[i] = (float)(P.f0[i] * s);
    P.fs[m + i] = (float)P.f0[m + i];
    P.fs[2 * m + i] = (float)P.f0[2 * m + i];
    P.fs[3 * m + i] = (float)(P.f0[3 * m + i] * s);
    P.fs[4 * m + i] = (float)(P.f0[4 * m + i] * s * s);
  }
  for (int j = t; j < n; j += kThreads) {
    const double s = e[j];
    P.gs[j] = (float)(P.g0[j] * s);
    P.gs[n + j] = (float)P.g0[n + j];
    P.gs[2 * n + j] = (float)P.g0[2 * n + j];
    P.gs[3 * n + j] = (float)(P.g0[3 * n + j] * s);
    P.gs[4 * n + j] = (float)(P.g0[4 * n + j] * s * s);
  }
  __syncthreads();
  // ---- K = I + G (lower triangle, Q x Q, identity on the padding) ----
  double *K = ws;
  double *X = ws + (size_t)Q * Q;
  double *Dinv = X + (size_t)Q * Q;
  for (int i = 0; i < Q; ++i)
    for (int j = t; j <= i; j += kThreads) K[(size_t)i * Q + j] = i == j ? 1.0 : 0.0;
  __syncthreads();
  const bool tall = m >= n;
  const int kdim = tall ? m : n;
  const int nt = (q + kGramTB - 1) / kGramTB;
  GramStage &gst = *reinterpret_cast<GramStage *>(lds);
  for (int tp = 0; tp < nt * (nt + 1) / 2; ++tp) {
    int ti, tj;
    tri_index(tp, &ti, &tj);
    for (int k0 = 0; k0 < kdim; k0 += 2048) {
      const int k1 = min(kdim, k0 + 2048);
      auto out = [&](int r, int c, float v) {
        const int gi = ti * kGramTB + r, gj = tj * kGramTB + c;
        if (gi < q && gj <= gi) K[(size_t)gi * Q + gj] += (double)v;
      };
      if (tall) gram_tile_f32<true>(A, m, n, ld, ti, tj, k0, k1, gst, out);
      else gram_tile_f32<false>(A, m, n, ld, ti, tj, k0, k1, gst, out);
      __syncthreads();
    }
  }
  // ---- blocked Cholesky ----
  const int nbt = Q / NB;
  CholLds &cl = *reinterpret_cast<CholLds *>(lds);
  F64Stage &fst = *reinterpret_cast<F64Stage *>(lds);
  for (int kb = 0; kb < nbt; ++kb) {
    potrf_diag(K, Q, kb, Dinv, &P.bad, cl);
    for (int ib = kb + 1; ib < nbt; ++ib) trsm_tile(K, Q, kb, ib, Dinv, fst);
    __syncthreads();
    for (int I = kb + 1; I < nbt; ++I)
      for (int J = kb + 1; J <= I; ++J) syrk_tile(K, Q, kb, I, J, fst);
    __syncthreads();
  }
  // ---- L^{-1} (right-looking blocks), then K^{-1} ----
  trtri_init_rows(X, Q, 0, Q);
  __syncthreads();
  for (int i = 0; i < nbt; ++i) {
    for (int j = 0; j <= i; ++j) trtri_scale_tile(Dinv, X, Q, i, j, fst);
    __syncthreads();
    for (int r = i + 1; r < nbt; ++r)
      for (int j = 0; j <= i; ++j) trtri_update_tile(K, X, Q, i, r, j, fst);
    __syncthreads();
  }
  for (int i = 0; i < q; ++i)
    for (int j = t; j < P.ldk; j += kThreads) P.Kinv[(size_t)i * P.ldk + j] = 0.0f;
  __syncthreads();
  for (int I = 0; I < nbt; ++I)
    for (int J = 0; J <= I; ++J) kinv_tile<float>(X, Q, nbt, q, P.Kinv, P.ldk, I, J, fst);
  __syncthreads();
  // ---- initial state (Algorithm 1 starts from zero) ----
  const size_t nvec = 5 * (size_t)P.ldn + 5 * (size_t)P.ldm + (size_t)P.ldk;
  for (size_t i = t; i < nvec; i += kThreads) P.vec[i] = 0.0f;
  if (t == 0) {
    P.rho = P.rho0;
    P.rescale = 1.0;
    P.k = P.l = P.u = 0;
    P.status = -1;
    P.setup_done = 1;
  }
  __syncthreads();
}

// --------------------------------------------------------------------------
// iterations of one problem
// --------------------------------------------------------------------------
__device__ void wg_iterate(BProb &P, char *lds, WgShared &sh, int budget) {
  const int m = P.m, n = P.n, ld = P.ld, q = P.q;
  const int t = threadIdx.x;
  float *x = P.vec, *xt = x + P.ldn, *xh = xt + P.ldn, *mu = xh + P.ldn, *cx = mu + P.ldn;
  float *y = cx + P.ldn, *yt = y + P.ldm, *yh = yt + P.ldm, *nu = yh + P.ldm, *dy = nu + P.ldm;
  float *rhs = dy + P.ldm;
  const float *fa = P.fs, *fb = fa + m, *fc = fb + m, *fd = fc + m, *fe = fd + m;
  const float *ga = P.gs, *gb = ga + n, *gc = gb + n, *gd = gc + n, *ge = gd + n;
  float *vs = reinterpret_cast<float *>(lds);
  const float alpha = (float)P.alpha;
  const bool tall = m >= n;
  for (int it = 0; it < budget; ++it) {
    const float rho = (float)P.rho;
    const float resc = (float)P.rescale;
    // ---- prox, half-step duals, relaxation (Alg. 1, Sections 3.2-3.3) ----
    double cmu = 0.0, cyh = 0.0;
    for (int j = t; j < n; j += kThreads) {
      float vt = xt[j];
      if (resc != 1.0f) {
        vt *= resc;
        xt[j] = vt;
      }
      const float v = x[j], arg = v - vt;
      const float h = prox_param<float>(P.gh[j], ga[j], gb[j], gc[j], gd[j], ge[j], arg, rho);
      const float du = -rho * (h - arg);
      xh[j] = h;
      mu[j] = du;
      cx[j] = alpha * h + (1.0f - alpha) * v + vt;
      cmu += (double)du * (double)du;
    }
    for (int i = t; i < m; i += kThreads) {
      float vt = yt[i];
      if (resc != 1.0f) {
        vt *= resc;
        yt[i] = vt;
      }
      const float v = y[i], arg = v - vt;
      const float h = prox_param<float>(P.fh[i], fa[i], fb[i], fc[i], fd[i], fe[i], arg, rho);
      yh[i] = h;
      nu[i] = -rho * (h - arg);
      dy[i] = alpha * h + (1.0f - alpha) * v + vt;
      cyh += (double)h * (double)h;
    }
    const double mu2 = block_sum(cmu, sh.bs);
    const double yh2 = block_sum(cyh, sh.bs);
    __syncthreads();
    // ---- projection (Section 3.5) with residual sums ----
    double pri2, dual2;
    if (tall) {
      dual2 = wg_gemv_t<false, 2, float>(P.A, m, n, ld, dy, nu, lds, sh, [&](int j, double w, double s) {
        rhs[j] = (float)((double)cx[j] + w);
        const double r = s + (double)mu[j];
        return r * r;
      });
      __syncthreads();
      wg_gemv_n<false, 1, float>(P.Kinv, q, q, P.ldk, rhs, rhs, vs, sh, [&](int j, double v, double) {
        const float xv = (float)v;
        x[j] = xv;
        xt[j] = cx[j] - xv;
        return 0.0;
      });
      __syncthreads();
      pri2 = wg_gemv_n<false, 2, float>(P.A, m, n, ld, x, xh, vs, sh, [&](int i, double yv, double tv) {
        const float yf = (float)yv;
        y[i] = yf;
        yt[i] = dy[i] - yf;
        const double r = tv - (double)yh[i];
        return r * r;
      });
    } else {
      pri2 = wg_gemv_n<false, 2, float>(P.A, m, n, ld, cx, xh, vs, sh, [&](int i, double u, double tv) {
        rhs[i] = (float)(u - (double)dy[i]);
        const double r = tv - (double)yh[i];
        return r * r;
      });
      __syncthreads();
      wg_gemv_n<false, 1, float>(P.Kinv, q, q, P.ldk, rhs, rhs, vs, sh, [&](int i, double z, double) {
        const float yf = (float)((double)dy[i] + z);
        y[i] = yf;
        yt[i] = dy[i] - yf;
        return 0.0;
      });
      __syncthreads();
      dual2 = wg_gemv_t<false, 2, float>(P.A, m, n, ld, yt, nu, lds, sh, [&](int j, double z, double s) {
        const float xf = (float)((double)cx[j] + z);
        x[j] = xf;
        xt[j] = cx[j] - xf;
        const double r = s + (double)mu[j];
        return r * r;
      });
    }
    // ---- stopping test and Algorithm 3 (thread 0 holds the sums) ----
    if (t == 0) {
      const double r_pri = sqrt(pri2), r_dual = sqrt(dual2);
      const double eps_pri = P.eps_abs + P.eps_rel * sqrt(yh2);
      const double eps_dual = P.eps_abs + P.eps_rel * sqrt(mu2);
      P.r_pri = r_pri;
      P.r_dual = r_dual;
      P.eps_pri = eps_pri;
      P.eps_dual = eps_dual;
      const int k = P.k;
      double rescale = 1.0;
      int status = -1;
      if (!isfinite(r_pri) || !isfinite(r_dual)) {
        status = POGS_NUMERICAL;
      } else if (r_pri < eps_pri && r_dual < eps_dual) {
        status = POGS_CONVERGED;
      } else {
        if (P.adaptive) {
          const double r0 = P.rho;
          double r1 = r0;
          if (r_dual < eps_dual && P.tau * k > P.l) {
            r1 = P.delta * r0;
            P.u = k;
          } else if (r_pri < eps_pri && P.tau * k > P.u) {
            r1 = r0 / P.delta;
            P.l = k;
          }
          if (r1 != r0) {
            rescale = r0 / r1;
            P.rho = r1;
          }
        }
        if (k + 1 >= P.max_iter) status = POGS_MAXITER;
      }
      P.rescale = rescale;
      P.k = k + 1;
      P.status = status;
      sh.done = status >= 0;
    }
    __syncthreads();
    const bool stop = sh.done != 0;
    __syncthreads();
    if (stop) break;
  }
}

// Half-step tuple in the original variables and the objective (Section 5).
__device__ void wg_finish(BProb &P, WgShared &sh) {
  const int m = P.m, n = P.n;
  const int t = threadIdx.x;
  const float *xh = P.vec + 2 * P.ldn, *mu = P.vec + 3 * P.ldn;
  const float *yh = P.vec + 5 * P.ldn + 2 * P.ldm, *nu = P.vec + 5 * P.ldn + 3 * P.ldm;
  float *ox = P.out, *oy = ox + n, *omu = oy + m, *onu = omu + n;
  double c = 0.0;
  for (int j = t; j < n; j += kThreads) {
    const double xv = P.E[j] * (double)xh[j];
    ox[j] = (float)xv;
    omu[j] = (float)((double)mu[j] / P.E[j]);
    c += fn_value(P.gh[j], P.g0[j], P.g0[n + j], P.g0[2 * n + j], P.g0[3 * n + j], P.g0[4 * n + j], xv);
  }
  for (int i = t; i < m; i += kThreads) {
    const double yv = (double)yh[i] / P.D[i];
    oy[i] = (float)yv;
    onu[i] = (float)(P.D[i] * (double)nu[i]);
    c += fn_value(P.fh[i], P.f0[i], P.f0[m + i], P.f0[2 * m + i], P.f0[3 * m + i], P.f0[4 * m + i], yv);
  }
  const double tot = block_sum(c, sh.bs);
  if (t == 0) P.optval = tot;
  __syncthreads();
}

}  // namespace

__global__ __launch_bounds__(kThreads) void batch_kernel(BProb *probs, const int *order, int count, unsigned *next,
                                                         double *scratch, size_t slot_doubles, int budget) {
  extern __shared__ __align__(16) char lds[];
  __shared__ WgShared sh;
  double *ws = scratch + (size_t)blockIdx.x * slot_doubles;
  for (;;) {
    if (threadIdx.x == 0) sh.idx = (int)atomicAdd(next, 1u);
    __syncthreads();
    const int idx = sh.idx;
    __syncthreads();
    if (idx >= count) break;
    BProb &P = probs[order[idx]];
    if (P.status >= 0 && P.setup_done) continue;  // already finished
    if (!P.setup_done) wg_setup(P, ws, lds, sh);
    if (P.bad) {
      if (threadIdx.x == 0) P.status = POGS_NUMERICAL;
      __syncthreads();
      continue;
    }
    wg_iterate(P, lds, sh, budget);
    if (P.status >= 0) wg_finish(P, sh);
  }
}

size_t batch_slot_doubles(int Qmax) {
  const size_t Q = (size_t)round_up(std::max(Qmax, 1), 64);
  return 2 * Q * Q + Q * 64;
}

size_t batch_lds_bytes(int max_n) {
  const size_t vec = 2 * (size_t)round_up(std::max(max_n, 1), 64) * sizeof(double);
  const size_t a = std::max(sizeof(CholLds), vec), b = std::max(sizeof(GramStage), sizeof(F64Stage));
  return std::max(std::max(a, b), sizeof(RedBuf));
}

void launch_batch(BProb *probs, const int *order, int count, unsigned *next, double *scratch, size_t slot_doubles,
                  int slots, int max_n, int iter_budget, hipStream_t s) {
  const size_t lds = batch_lds_bytes(max_n);
  hipLaunchKernelGGL(batch_kernel, dim3(slots), dim3(kThreads), lds, s, probs, order, count, next, scratch,
                     slot_doubles, iter_budget);
}

}  // namespace pogs
