// Lambda path: R problems that share the scaled matrix A^ = D A E and its
// cached K^{-1} (m >= n), iterated together.  The R right-hand sides of each
// pass over A are stacked into one matrix, so the two passes and the solve are
// f32 MFMA matrix products (one read of A per pass for all R problems), with
// K split across workgroups and the split partials summed in float64 in a
// fixed order.  Every problem keeps its own rho, Algorithm 3 markers and stop
// test (a stopped problem's state is frozen while the others continue).
//
// Per iteration (columns r < R of every state matrix):
//   prox    : x_h, y_h, mu_h, nu_h, relaxed c, d per column     (Alg. 1, 3.2, 3.3)
//   pass 1  : [W | S] = A^T [Dy | Nu]  -> Rhs = Cx + W, ||S + Mu||^2 per column
//   solve   : X = K^{-1} Rhs, Xt = Cx - X
//   pass 2  : [Y | T] = A [X | Xh]     -> Yt = Dy - Y, ||T - Yh||^2 per column
//   control : per-column stopping test and Algorithm 3                (3.4, 4.3)
#include "factor.hpp"
#include "path.hpp"
#include "prox.hpp"

namespace pogs {

namespace {

// prox over rows [0, n) (x side) then [n, n + m) (y side); block = 64 columns x 4 row groups.
__global__ __launch_bounds__(256) void path_prox_kernel(PathArgs p) {
  __shared__ double red[2][4][64];
  if (*p.all_done) return;
  const int col = blockIdx.x * 64 + (threadIdx.x & 63);
  const int rg = threadIdx.x >> 6;
  const bool xs = (int)blockIdx.y < p.nbx;
  const int blk = xs ? blockIdx.y : blockIdx.y - p.nbx;
  const int len = xs ? p.n : p.m;
  const int r0 = blk * p.rows_per_block;
  const int r1 = min(len, r0 + p.rows_per_block);
  double acc = 0.0;
  if (col < p.R && !p.done[col]) {
    const float rho = (float)p.rho[col];
    const float resc = (float)p.rescale[col];
    const float alpha = p.alpha;
    const int Rp = p.Rp;
    for (int i = r0 + rg; i < r1; i += 4) {
      const size_t e = (size_t)i * Rp + col;
      if (xs) {
        float vt = p.Xt[e];
        if (resc != 1.0f) {
          vt *= resc;
          p.Xt[e] = vt;
        }
        const size_t e2 = (size_t)i * 2 * Rp + col;
        const float v = p.XX[e2], arg = v - vt;
        const float h = prox_param<float>(p.gh[e], p.ga[e], p.gb[e], p.gc[e], p.gd[e], p.ge[e], arg, rho);
        const float du = -rho * (h - arg);
        p.XX[e2 + Rp] = h;
        p.Mu[e] = du;
        p.Cx[e] = alpha * h + (1.0f - alpha) * v + vt;
        acc += (double)du * (double)du;
      } else {
        float vt = p.Yt[e];
        if (resc != 1.0f) {
          vt *= resc;
          p.Yt[e] = vt;
        }
        const float v = p.Y[e], arg = v - vt;
        const float h = prox_param<float>(p.fh[e], p.fa[e], p.fb[e], p.fc[e], p.fd[e], p.fe[e], arg, rho);
        p.Yh[e] = h;
        const size_t e2 = (size_t)i * 2 * Rp + col;
        p.DN[e2 + Rp] = -rho * (h - arg);
        p.DN[e2] = alpha * h + (1.0f - alpha) * v + vt;
        acc += (double)h * (double)h;
      }
    }
  }
  red[0][rg][threadIdx.x & 63] = acc;
  __syncthreads();
  if (threadIdx.x < 64 && col < p.R) {
    const double s = (red[0][0][threadIdx.x] + red[0][1][threadIdx.x]) + (red[0][2][threadIdx.x] + red[0][3][threadIdx.x]);
    (xs ? p.s_mu : p.s_yh)[(size_t)blk * p.Rp + col] = s;
  }
}

// Split-K partial product of one 128 x 128 output tile:
// part[split][i][j] = sum_{k in split} opA(i, k) B(k, j).
template <bool A_T>
__global__ __launch_bounds__(512) void path_gemm_kernel(const float *A, int lda, int M, const float *B, int ldb, int N,
                                                        int K, int kchunk, float *part, const int *all_done) {
  __shared__ GemmStage st[2];
  if (*all_done) return;
  const int i0 = blockIdx.x * kGramTB, j0 = blockIdx.y * kGramTB;
  const int k0 = blockIdx.z * kchunk, k1 = min(K, k0 + kchunk);
  float *out = part + (size_t)blockIdx.z * M * N;
  gemm_tile_f32<A_T>(A, lda, M, B, ldb, N, i0, j0, k0, k1, st, [&](int r, int c, float v) {
    const int gi = i0 + r, gj = j0 + c;
    if (gi < M && gj < N) out[(size_t)gi * N + gj] = v;
  });
}

// Sum split partials of an M x N product in split order (float64); hand each
// element to the epilogue; per-column sums of the epilogue's return value per
// row block go to slots[block][col - col_off] for col >= col_off.
template <class Epi>
__global__ __launch_bounds__(256) void path_reduce_kernel(PathArgs p, const float *part, int splits, int M, int N,
                                                          int rows_per_block, Epi epi) {
  __shared__ double red[4][64];
  if (*p.all_done) return;
  const int col = blockIdx.x * 64 + (threadIdx.x & 63);
  const int rg = threadIdx.x >> 6;
  const int r0 = blockIdx.y * rows_per_block;
  const int r1 = min(M, r0 + rows_per_block);
  double acc = 0.0;
  if (col < N) {
    for (int i = r0 + rg; i < r1; i += 4) {
      // eight split partials loaded together, then added in split order (the
      // same bits as one at a time; a loop with a run-time trip count would
      // wait for each load before issuing the next)
      double v = 0.0;
      int s = 0;
      for (; s + 8 <= splits; s += 8) {
        float t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = part[((size_t)(s + u) * M + i) * N + col];
#pragma unroll
        for (int u = 0; u < 8; ++u) v += (double)t[u];
      }
      for (; s < splits; ++s) v += (double)part[((size_t)s * M + i) * N + col];
      acc += epi(p, i, col, v);
    }
  }
  red[rg][threadIdx.x & 63] = acc;
  __syncthreads();
  if (threadIdx.x < 64 && col < N) {
    const double s = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
    epi.slot(p, blockIdx.y, col, s);
  }
}

struct EpiPass1 {  // [W | S] = A^T [Dy | Nu]
  __device__ double operator()(const PathArgs &p, int j, int c, double v) const {
    const int Rp = p.Rp;
    if (c < Rp) {
      if (c < p.R && !p.done[c]) p.Rhs[(size_t)j * Rp + c] = (float)((double)p.Cx[(size_t)j * Rp + c] + v);
      return 0.0;
    }
    const int r = c - Rp;
    if (r >= p.R || p.done[r]) return 0.0;
    const double d = v + (double)p.Mu[(size_t)j * Rp + r];
    return d * d;
  }
  __device__ void slot(const PathArgs &p, int b, int c, double s) const {
    if (c >= p.Rp && c - p.Rp < p.R) p.s_dual[(size_t)b * p.Rp + c - p.Rp] = s;
  }
};

struct EpiSolve {  // X = K^{-1} Rhs
  __device__ double operator()(const PathArgs &p, int j, int c, double v) const {
    if (c < p.R && !p.done[c]) {
      const float xv = (float)v;
      p.XX[(size_t)j * 2 * p.Rp + c] = xv;
      p.Xt[(size_t)j * p.Rp + c] = p.Cx[(size_t)j * p.Rp + c] - xv;
    }
    return 0.0;
  }
  __device__ void slot(const PathArgs &, int, int, double) const {}
};

struct EpiPass2 {  // [Y | T] = A [X | Xh]
  __device__ double operator()(const PathArgs &p, int i, int c, double v) const {
    const int Rp = p.Rp;
    if (c < Rp) {
      if (c < p.R && !p.done[c]) {
        const float yv = (float)v;
        p.Y[(size_t)i * Rp + c] = yv;
        p.Yt[(size_t)i * Rp + c] = p.DN[(size_t)i * 2 * Rp + c] - yv;
      }
      return 0.0;
    }
    const int r = c - Rp;
    if (r >= p.R || p.done[r]) return 0.0;
    const double d = v - (double)p.Yh[(size_t)i * Rp + r];
    return d * d;
  }
  __device__ void slot(const PathArgs &p, int b, int c, double s) const {
    if (c >= p.Rp && c - p.Rp < p.R) p.s_pri[(size_t)b * p.Rp + c - p.Rp] = s;
  }
};

// One workgroup per problem r: its four residual sums over the block slots
// (a strided share per thread, then a fixed-order tree), then thread 0 runs
// the stopping test and Algorithm 3 on its own residuals.
__global__ __launch_bounds__(256) void path_control_kernel(PathArgs p) {
  __shared__ double scratch[256 / kWave];
  const int r = blockIdx.x;
  if (*p.all_done || p.done[r]) return;  // the same for the whole workgroup
  double mu2 = 0.0, yh2 = 0.0, pri2 = 0.0, dual2 = 0.0;
  for (int b = threadIdx.x; b < p.nbx; b += blockDim.x) mu2 += p.s_mu[(size_t)b * p.Rp + r];
  for (int b = threadIdx.x; b < p.nby; b += blockDim.x) yh2 += p.s_yh[(size_t)b * p.Rp + r];
  for (int b = threadIdx.x; b < p.nb_pri; b += blockDim.x) pri2 += p.s_pri[(size_t)b * p.Rp + r];
  for (int b = threadIdx.x; b < p.nb_dual; b += blockDim.x) dual2 += p.s_dual[(size_t)b * p.Rp + r];
  mu2 = block_sum(mu2, scratch);
  yh2 = block_sum(yh2, scratch);
  pri2 = block_sum(pri2, scratch);
  dual2 = block_sum(dual2, scratch);
  if (threadIdx.x != 0) return;
  const double r_pri = sqrt(pri2), r_dual = sqrt(dual2);
  const double eps_pri = p.eps_abs + p.eps_rel * sqrt(yh2);
  const double eps_dual = p.eps_abs + p.eps_rel * sqrt(mu2);
  p.r_pri[r] = r_pri;
  p.r_dual[r] = r_dual;
  p.eps_pri[r] = eps_pri;
  p.eps_dual[r] = eps_dual;
  const int k = p.iters[r];
  double rescale = 1.0;
  int status = -1;
  if (!isfinite(r_pri) || !isfinite(r_dual)) {
    status = POGS_NUMERICAL;
  } else if (r_pri < eps_pri && r_dual < eps_dual) {
    status = POGS_CONVERGED;
  } else {
    if (p.adaptive) {
      const double r0 = p.rho[r];
      double r1 = r0;
      if (r_dual < eps_dual && p.tau * k > p.l[r]) {
        r1 = p.delta * r0;
        p.u[r] = k;
      } else if (r_pri < eps_pri && p.tau * k > p.u[r]) {
        r1 = r0 / p.delta;
        p.l[r] = k;
      }
      if (r1 != r0) {
        rescale = r0 / r1;
        p.rho[r] = r1;
      }
    }
    if (k + 1 >= p.max_iter) status = POGS_MAXITER;
  }
  p.rescale[r] = rescale;
  p.iters[r] = k + 1;
  if (status >= 0) {
    p.status[r] = status;
    p.done[r] = 1;
  }
}

// Sets all_done once every problem has stopped (after the control step).
__global__ void path_alldone_kernel(PathArgs p) {
  __shared__ int live;
  if (*p.all_done) return;
  if (threadIdx.x == 0) live = 0;
  __syncthreads();
  for (int r = threadIdx.x; r < p.R; r += blockDim.x)
    if (!p.done[r]) atomicAdd(&live, 1);
  __syncthreads();
  if (threadIdx.x == 0 && live == 0) *p.all_done = 1;
}

// f^ and g^ parameters per problem: f^(y) = f(y / D), g^(x) = g(E x).
__global__ void path_scale_fn_kernel(const double *src, const uint8_t *hsrc, int len, int Rp, const double *scale,
                                     bool divide, uint8_t *h, float *a, float *b, float *c, float *d, float *e) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t tot = (size_t)len * Rp;
  if (idx >= tot) return;
  const int i = (int)(idx / Rp);
  const double s = divide ? 1.0 / scale[i] : scale[i];
  h[idx] = hsrc[idx];
  a[idx] = (float)(src[idx] * s);
  b[idx] = (float)src[tot + idx];
  c[idx] = (float)src[2 * tot + idx];
  d[idx] = (float)(src[3 * tot + idx] * s);
  e[idx] = (float)(src[4 * tot + idx] * s * s);
}

// Half-step tuple of problem r in the original variables, and f(y) + g(x).
__global__ __launch_bounds__(256) void path_unscale_kernel(PathArgs p, const double *D, const double *E,
                                                           const double *f0, const uint8_t *fh0, const double *g0,
                                                           const uint8_t *gh0, float *out, double *obj) {
  __shared__ double bs[4];
  const int r = blockIdx.x;
  const int m = p.m, n = p.n, Rp = p.Rp;
  const size_t tf = (size_t)m * Rp, tg = (size_t)n * Rp;
  float *ox = out + (size_t)r * 2 * (m + n), *oy = ox + n, *omu = oy + m, *onu = omu + n;
  double c = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const size_t e = (size_t)j * Rp + r;
    const double xv = E[j] * (double)p.XX[(size_t)j * 2 * Rp + Rp + r];
    ox[j] = (float)xv;
    omu[j] = (float)((double)p.Mu[e] / E[j]);
    c += fn_value(gh0[e], g0[e], g0[tg + e], g0[2 * tg + e], g0[3 * tg + e], g0[4 * tg + e], xv);
  }
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const size_t e = (size_t)i * Rp + r;
    const double yv = (double)p.Yh[e] / D[i];
    oy[i] = (float)yv;
    onu[i] = (float)(D[i] * (double)p.DN[(size_t)i * 2 * Rp + Rp + r]);
    c += fn_value(fh0[e], f0[e], f0[tf + e], f0[2 * tf + e], f0[3 * tf + e], f0[4 * tf + e], yv);
  }
  const double tot = block_sum(c, bs);
  if (threadIdx.x == 0) obj[r] = tot;
}

// Splits of K: about two workgroups per CU at most, chunks of at least 256
// unless that leaves fewer than 128 workgroups (a small product such as the
// solve), then chunks down to 64.
int gemm_splits(int M, int N, int K) {
  const int64_t tiles = cdiv(M, kGramTB) * cdiv(N, kGramTB);
  const int64_t want = std::max<int64_t>(cdiv(K, 256), std::min<int64_t>(cdiv(128, tiles), cdiv(K, 64)));
  return (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(512, tiles), want));
}

template <bool A_T>
void gemm(const float *A, int lda, int M, const float *B, int ldb, int N, int K, float *part, int splits,
          const int *all_done, hipStream_t s) {
  const int kchunk = (int)round_up(cdiv(K, splits), kGemmKC);
  const int sp = (int)cdiv(K, kchunk);
  dim3 grid(cdiv(M, kGramTB), cdiv(N, kGramTB), sp);
  hipLaunchKernelGGL(path_gemm_kernel<A_T>, grid, dim3(512), 0, s, A, lda, M, B, ldb, N, K, kchunk, part, all_done);
}

int actual_splits(int K, int splits) {
  const int kchunk = (int)round_up(cdiv(K, splits), kGemmKC);
  return (int)cdiv(K, kchunk);
}

}  // namespace

void path_geometry(PathArgs *p, int *s1, int *s2, int *s3) {
  const int n = p->n, m = p->m, N2 = 2 * p->Rp;
  *s1 = actual_splits(m, gemm_splits(n, N2, m));
  *s2 = actual_splits(n, gemm_splits(n, p->Rp, n));
  *s3 = actual_splits(n, gemm_splits(m, N2, n));
}

void launch_path_scale_fn(const double *src, const uint8_t *hsrc, int len, int Rp, const double *scale, bool divide,
                          uint8_t *h, float *a, float *b, float *c, float *d, float *e, hipStream_t s) {
  const size_t tot = (size_t)len * Rp;
  hipLaunchKernelGGL(path_scale_fn_kernel, dim3(cdiv(tot, 256)), dim3(256), 0, s, src, hsrc, len, Rp, scale, divide,
                     h, a, b, c, d, e);
}

void launch_path_iteration(const PathArgs &p, float *part, hipStream_t s) {
  const int n = p.n, m = p.m, Rp = p.Rp, N2 = 2 * Rp;
  const dim3 cols(cdiv(N2, 64));
  hipLaunchKernelGGL(path_prox_kernel, dim3(cdiv(p.R, 64), p.nbx + p.nby), dim3(256), 0, s, p);
  // pass 1: [W | S] = A^T [Dy | Nu]   (A stored m x n: A_T with K = m)
  const int s1 = gemm_splits(n, N2, m);
  gemm<true>(p.A, p.ld, n, p.DN, N2, N2, m, part, s1, p.all_done, s);
  hipLaunchKernelGGL(path_reduce_kernel<EpiPass1>, dim3(cols.x, p.nb_dual), dim3(256), 0, s, p, (const float *)part,
                     actual_splits(m, s1), n, N2, p.rows_per_block, EpiPass1{});
  // solve: X = K^{-1} Rhs
  const int s2 = gemm_splits(n, Rp, n);
  gemm<false>(p.Kinv, p.ldk, n, p.Rhs, Rp, Rp, n, part, s2, p.all_done, s);
  hipLaunchKernelGGL(path_reduce_kernel<EpiSolve>, dim3(cdiv(Rp, 64), p.nb_dual), dim3(256), 0, s, p,
                     (const float *)part, actual_splits(n, s2), n, Rp, p.rows_per_block, EpiSolve{});
  // pass 2: [Y | T] = A [X | Xh]
  const int s3 = gemm_splits(m, N2, n);
  gemm<false>(p.A, p.ld, m, p.XX, N2, N2, n, part, s3, p.all_done, s);
  hipLaunchKernelGGL(path_reduce_kernel<EpiPass2>, dim3(cols.x, p.nb_pri), dim3(256), 0, s, p, (const float *)part,
                     actual_splits(n, s3), m, N2, p.rows_per_block, EpiPass2{});
  hipLaunchKernelGGL(path_control_kernel, dim3(p.R), dim3(256), 0, s, p);
  hipLaunchKernelGGL(path_alldone_kernel, dim3(1), dim3(256), 0, s, p);
}

void launch_path_unscale(const PathArgs &p, const double *D, const double *E, const double *f0, const uint8_t *fh0,
                         const double *g0, const uint8_t *gh0, float *out, double *obj, hipStream_t s) {
  hipLaunchKernelGGL(path_unscale_kernel, dim3(p.R), dim3(256), 0, s, p, D, E, f0, fh0, g0, gh0, out, obj);
}

size_t path_part_floats(int m, int n, int Rp) {
  PathArgs p{};
  p.m = m;
  p.n = n;
  p.Rp = Rp;
  int s1, s2, s3;
  path_geometry(&p, &s1, &s2, &s3);
  const size_t N2 = 2 * (size_t)Rp;
  return std::max(std::max((size_t)s1 * n * N2, (size_t)s2 * n * Rp), (size_t)s3 * m * N2);
}

}  // namespace pogs
