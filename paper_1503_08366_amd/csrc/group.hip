// Grouped launches over many problems (see group.hpp): one kernel per phase,
// each workgroup taking the work item at its block index and running the
// phase's device body on that problem.
#include "group.hpp"
#include "iter.hpp"
#include "setup.hpp"

namespace pogs {

namespace {

#define GROUP_ITEM()                                \
  const GItem w = items[blockIdx.x];                \
  const GProb &P = probs[w.prob];                   \
  const Blk b{w.x, w.y, w.nx, w.ny};

// Row-major float32 input -> padded A (rows [b.x rows, (b.x + 1) rows)),
// counting non-finite entries; the first workgroup also sets e = 1 for the
// first Sinkhorn-Knopp sweep.
__device__ __forceinline__ void layout_rows_body(const Blk &b, const GProb &P) {
  const int m = P.it.m, n = P.it.n, ld = P.it.ld;
  float *dst = const_cast<float *>(P.it.A);
  unsigned nbad = 0;
  const int r0 = b.x * P.lay_rows, r1 = min(m, r0 + P.lay_rows);
  for (int r = r0; r < r1; ++r)
    for (int c = threadIdx.x; c < ld; c += blockDim.x) {
      float v = 0.f;
      if (c < n) {
        v = P.raw[(size_t)r * P.lda + c];
        if (!isfinite(v)) ++nbad;
      }
      dst[(size_t)r * ld + c] = v;
    }
  if (nbad) atomicAdd(P.flags, nbad);
  if (b.x == 0 && b.y == 0)
    for (int j = threadIdx.x; j < n; j += blockDim.x) P.e[j] = 1.0;
}

__global__ __launch_bounds__(256) void g_layout_rows(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  layout_rows_body(b, P);
}

__global__ __launch_bounds__(256) void g_layout_tiles(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  layout_body<float, float>(b, P.raw, 1, P.lda, P.it.m, P.it.n, const_cast<float *>(P.it.A), P.it.ld, P.flags);
  if (b.x == 0 && b.y == 0)
    for (int j = threadIdx.x; j < P.it.n; j += blockDim.x) P.e[j] = 1.0;
}

template <int U>
__global__ __launch_bounds__(kBlock) void g_eq_sweep(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  equil_sweep_body<U, 4>(b, P.it.A, P.it.m, P.it.n, P.it.ld, P.eq_rps, P.e, P.d, P.eq_part, P.eq_ncolp, P.nf,
                         P.gamma_m);
}

__device__ __forceinline__ EqArgs eq_args(const GProb &P) {
  EqArgs a;
  a.d = P.d;
  a.e = P.e;
  a.colsum = nullptr;
  a.slots = P.eq_slots;
  a.fro2 = nullptr;
  a.gamma_m = P.gamma_m;
  a.gamma_n = P.gamma_n;
  a.mf = P.mf;
  a.nf = P.nf;
  return a;
}

__global__ __launch_bounds__(kBlock) void g_eq_colfinish(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  EpiEqCol e{eq_args(P)};
  gemv_t_finish_body<1, EpiEqCol>(b, P.it.n, P.eq_nsplit, P.eq_part, P.eq_ncolp, e);
}

__global__ __launch_bounds__(256) void g_eq_normalize(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  const int m = P.it.m, n = P.it.n;
  if (P.equil_iters <= 0) {
    const int i = b.x * 256 + threadIdx.x;
    if (i < m) P.D[i] = 1.0;
    else if (i < m + n) P.E[i - m] = 1.0;
    return;
  }
  equil_finish_body(b, P.d, P.e, P.eq_slots, (int)((n + kFinishCols - 1) / kFinishCols), m, n, P.it.q, P.D, P.E);
}

__global__ __launch_bounds__(256) void g_scale_matrix(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  scale_matrix_body<float>(b, const_cast<float *>(P.it.A), P.it.m, P.it.n, P.it.ld, P.D, P.E);
}

__global__ __launch_bounds__(kBlock) void g_scale_fn(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  const int m = P.it.m, n = P.it.n;
  if (b.y == 0) {
    const FnDev<float> &F = P.it.f;
    scale_fn_body<float>(b, P.fh0, P.f0, P.f0 + m, P.f0 + 2 * m, P.f0 + 3 * m, P.f0 + 4 * m, P.D, true, m,
                         const_cast<uint8_t *>(F.h), const_cast<float *>(F.a), const_cast<float *>(F.b),
                         const_cast<float *>(F.c), const_cast<float *>(F.d), const_cast<float *>(F.e));
  } else {
    const FnDev<float> &G = P.it.g;
    scale_fn_body<float>(b, P.gh0, P.g0, P.g0 + n, P.g0 + 2 * n, P.g0 + 3 * n, P.g0 + 4 * n, P.E, false, n,
                         const_cast<uint8_t *>(G.h), const_cast<float *>(G.a), const_cast<float *>(G.b),
                         const_cast<float *>(G.c), const_cast<float *>(G.d), const_cast<float *>(G.e));
  }
}

// K = I + G, one tile per workgroup, written as float64 into the lower
// triangle of K; the identity fills the padding up to Q.  The K range is
// summed in chunks of kGChunk in float32 (as the single-problem path does
// inside a split) and the chunks are added in float64 in order, so a long
// K range (m rows of a tall problem) does not accumulate in float32.
constexpr int kGChunk = 4096;
__global__ __launch_bounds__(256, 4) void g_gram(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  __shared__ GramStage st[2];
  int ti, tj;
  tri_index(b.x, &ti, &tj);
  const int m = P.it.m, n = P.it.n, Q = P.Q;
  const int kdim = P.tall ? m : n;
  double *K = P.K;
  for (int k0 = 0; k0 < kdim; k0 += kGChunk) {
    const int k1 = min(kdim, k0 + kGChunk);
    const bool first = k0 == 0;
    auto out = [&](int r, int c, float v) {
      const int gi = ti * kGramTB + r, gj = tj * kGramTB + c;
      if (gi < Q && gj <= gi) {
        double &dst = K[(size_t)gi * Q + gj];
        dst = (first ? (gi == gj ? 1.0 : 0.0) : dst) + (double)v;
      }
    };
    if (P.tall) gram_tile_f32<true>(P.it.A, m, n, P.it.ld, ti, tj, k0, k1, st, out);
    else gram_tile_f32<false>(P.it.A, m, n, P.it.ld, ti, tj, k0, k1, st, out);
  }
}

__global__ __launch_bounds__(256) void g_trtri_init(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  trtri_init_rows(P.X, P.Q, b.x * 32, min(P.Q, b.x * 32 + 32));
}

__global__ __launch_bounds__(256) void g_potrf0(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  (void)b;
  __shared__ CholLds s;
  potrf_diag(P.K, P.Q, 0, P.Dinv, P.flags + 1, s);
}

__global__ __launch_bounds__(256) void g_panel(const GProb *probs, const GItem *items, int kb) {
  GROUP_ITEM();
  factor_panel_body(b.x, P.K, P.X, P.Q, P.nbt, kb, P.Dinv);
}

__global__ __launch_bounds__(256) void g_update(const GProb *probs, const GItem *items, int kb) {
  GROUP_ITEM();
  factor_update_body(b.x, P.K, P.X, P.Q, P.nbt, kb, P.Dinv, P.flags + 1);
}

__global__ __launch_bounds__(256) void g_kinv(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  kinv_body<float>(b.x, P.X, P.Q, P.nbt, P.it.q, const_cast<float *>(P.it.Kinv), P.it.ldk);
}

// ---- iteration ---------------------------------------------------------
__device__ __forceinline__ IterArgs<float> iter_args(const GProb &P, int par) {
  IterArgs<float> p = P.it;
  p.par = par;
  return p;
}

__global__ __launch_bounds__(kBlock) void g_prox(const GProb *probs, const GItem *items, int par) {
  GROUP_ITEM();
  prox_body<float>(b, iter_args(P, par));
}

__global__ __launch_bounds__(kBlock) void g_pass1_t(const GProb *probs, const GItem *items, int par) {
  GROUP_ITEM();
  const IterArgs<float> p = iter_args(P, par);
  EpiTallPass1<float> e{{p}};
  gemv_t_body<float, float, 2, false>(b, p.A, p.m, p.n, p.ld, p.dy, p.nu, P.rps, p.part, P.ncolp, e);
}

template <int LPR, int RPT>
__global__ __launch_bounds__(kBlock) void g_pass1_w(const GProb *probs, const GItem *items, int par) {
  GROUP_ITEM();
  const IterArgs<float> p = iter_args(P, par);
  EpiWidePass1<float> e{{p}};
  gemv_n_body<float, float, 2, false, LPR, RPT>(b, p.A, p.m, p.n, p.ld, p.cx, p.xh, e);
}

__global__ __launch_bounds__(kBlock) void g_finish1(const GProb *probs, const GItem *items, int par) {
  GROUP_ITEM();
  const IterArgs<float> p = iter_args(P, par);
  EpiTallPass1<float> e{{p}};
  gemv_t_finish_body<2>(b, p.n, P.splits, p.part, P.ncolp, e);
}

// The solve's epilogue for either orientation (chosen per problem).
struct EpiSolveAny {
  IterArgs<float> p;
  int tall;
  __device__ bool skip() const { return p.ctrl->st[p.par].done != 0; }
  __device__ double row(int i, double z, double) const {
    if (tall) {
      const float xv = (float)z;
      p.x[i] = xv;
      p.xt[i] = p.cx[i] - xv;
    } else {
      const float yv = (float)((double)p.dy[i] + z);
      p.y[i] = yv;
      p.yt[i] = p.dy[i] - yv;
    }
    return 0.0;
  }
  __device__ void block_done(int, double) const {}
};

template <int LPR, int RPT>
__global__ __launch_bounds__(kBlock) void g_solve(const GProb *probs, const GItem *items, int par) {
  GROUP_ITEM();
  const IterArgs<float> p = iter_args(P, par);
  EpiSolveAny e{p, P.tall};
  gemv_n_body<float, float, 1, false, LPR, RPT>(b, p.Kinv, p.q, p.q, p.ldk, p.rhs, p.rhs, e);
}

template <int LPR, int RPT>
__global__ __launch_bounds__(kBlock) void g_pass2_t(const GProb *probs, const GItem *items, int par) {
  GROUP_ITEM();
  const IterArgs<float> p = iter_args(P, par);
  EpiTallPass2<float> e{{p}};
  gemv_n_body<float, float, 2, false, LPR, RPT>(b, p.A, p.m, p.n, p.ld, p.x, p.xh, e);
}

__global__ __launch_bounds__(kBlock) void g_pass2_w(const GProb *probs, const GItem *items, int par) {
  GROUP_ITEM();
  const IterArgs<float> p = iter_args(P, par);
  EpiWidePass2<float> e{{p}};
  gemv_t_body<float, float, 2, false>(b, p.A, p.m, p.n, p.ld, p.yt, p.nu, P.rps, p.part, P.ncolp, e);
}

__global__ __launch_bounds__(kBlock) void g_finish2(const GProb *probs, const GItem *items, int par) {
  GROUP_ITEM();
  const IterArgs<float> p = iter_args(P, par);
  EpiWidePass2<float> e{{p}};
  gemv_t_finish_body<2>(b, p.n, P.splits, p.part, P.ncolp, e);
}

__global__ __launch_bounds__(kBlock) void g_preview(const GProb *probs, const GItem *items, int par) {
  GROUP_ITEM();
  (void)b;
  control_preview_body<float>(iter_args(P, par), par);
}

__global__ __launch_bounds__(kBlock) void g_unscale(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  const IterArgs<float> p = iter_args(P, 0);
  const int m = p.m, n = p.n;
  const double *fa = P.f0, *ga = P.g0;
  float *o = P.out;
  unscale_body<float>(b, p, P.D, P.E, P.fh0, fa, fa + m, fa + 2 * m, fa + 3 * m, fa + 4 * m, P.gh0, ga, ga + n,
                      ga + 2 * n, ga + 3 * n, ga + 4 * n, o, o + n, o + n + m, o + 2 * n + m, P.obj_slots, P.obj,
                      P.obj_cnt);
}

__global__ __launch_bounds__(64) void g_init_state(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  (void)b;
  if (threadIdx.x != 0) return;
  Ctrl c{};
  c.eps_abs = P.eps_abs;
  c.eps_rel = P.eps_rel;
  c.alpha = P.alpha;
  c.delta = P.delta;
  c.tau = P.tau;
  c.max_iter = P.max_iter;
  c.adaptive = P.adaptive;
  for (int k = 0; k < 2; ++k) {  // iteration 0 reads st[1]: no stop test pending
    c.st[k].rho = P.rho0;
    c.st[k].rescale = 1.0;
  }
  *P.it.ctrl = c;
}

__global__ __launch_bounds__(64) void g_gather(const GProb *probs, const GItem *items) {
  GROUP_ITEM();
  (void)b;
  if (threadIdx.x != 0) return;
  GStatus s;
  s.st = P.it.ctrl->st[0];
  s.flags[0] = P.flags[0];
  s.flags[1] = P.flags[1];
  s.obj = *P.obj;
  *P.status = s;
}

#undef GROUP_ITEM

}  // namespace

void launch_group(int phase, const GProb *probs, const GItem *items, int count, int arg, hipStream_t s) {
  if (count <= 0) return;
  const dim3 grid(count), blk(256);
  switch (phase) {
    case G_LAYOUT_ROWS: hipLaunchKernelGGL(g_layout_rows, grid, blk, 0, s, probs, items); break;
    case G_LAYOUT_TILES: hipLaunchKernelGGL(g_layout_tiles, grid, blk, 0, s, probs, items); break;
    case G_EQ_SWEEP:
      switch (arg) {
        case 1: hipLaunchKernelGGL(g_eq_sweep<1>, grid, blk, 0, s, probs, items); break;
        case 2: hipLaunchKernelGGL(g_eq_sweep<2>, grid, blk, 0, s, probs, items); break;
        case 3: hipLaunchKernelGGL(g_eq_sweep<3>, grid, blk, 0, s, probs, items); break;
        default: hipLaunchKernelGGL(g_eq_sweep<4>, grid, blk, 0, s, probs, items); break;
      }
      break;
    case G_EQ_COLFINISH: hipLaunchKernelGGL(g_eq_colfinish, grid, blk, 0, s, probs, items); break;
    case G_EQ_NORMALIZE: hipLaunchKernelGGL(g_eq_normalize, grid, blk, 0, s, probs, items); break;
    case G_SCALE_MATRIX: hipLaunchKernelGGL(g_scale_matrix, grid, blk, 0, s, probs, items); break;
    case G_SCALE_FN: hipLaunchKernelGGL(g_scale_fn, grid, blk, 0, s, probs, items); break;
    case G_GRAM: hipLaunchKernelGGL(g_gram, grid, blk, 0, s, probs, items); break;
    case G_TRTRI_INIT: hipLaunchKernelGGL(g_trtri_init, grid, blk, 0, s, probs, items); break;
    case G_POTRF0: hipLaunchKernelGGL(g_potrf0, grid, blk, 0, s, probs, items); break;
    case G_PANEL: hipLaunchKernelGGL(g_panel, grid, blk, 0, s, probs, items, arg); break;
    case G_UPDATE: hipLaunchKernelGGL(g_update, grid, blk, 0, s, probs, items, arg); break;
    case G_KINV: hipLaunchKernelGGL(g_kinv, grid, blk, 0, s, probs, items); break;
    case G_PROX: hipLaunchKernelGGL(g_prox, grid, blk, 0, s, probs, items, arg); break;
    case G_PASS1_T: hipLaunchKernelGGL(g_pass1_t, grid, blk, 0, s, probs, items, arg); break;
    case G_PASS1_W64: hipLaunchKernelGGL((g_pass1_w<64, 4>), grid, blk, 0, s, probs, items, arg); break;
    case G_PASS1_W16: hipLaunchKernelGGL((g_pass1_w<16, 4>), grid, blk, 0, s, probs, items, arg); break;
    case G_FINISH1: hipLaunchKernelGGL(g_finish1, grid, blk, 0, s, probs, items, arg); break;
    case G_SOLVE64: hipLaunchKernelGGL((g_solve<64, 4>), grid, blk, 0, s, probs, items, arg); break;
    case G_SOLVE16: hipLaunchKernelGGL((g_solve<16, 4>), grid, blk, 0, s, probs, items, arg); break;
    case G_PASS2_T64: hipLaunchKernelGGL((g_pass2_t<64, 4>), grid, blk, 0, s, probs, items, arg); break;
    case G_PASS2_T16: hipLaunchKernelGGL((g_pass2_t<16, 4>), grid, blk, 0, s, probs, items, arg); break;
    case G_PASS2_W: hipLaunchKernelGGL(g_pass2_w, grid, blk, 0, s, probs, items, arg); break;
    case G_FINISH2: hipLaunchKernelGGL(g_finish2, grid, blk, 0, s, probs, items, arg); break;
    case G_PREVIEW: hipLaunchKernelGGL(g_preview, grid, blk, 0, s, probs, items, arg); break;
    case G_UNSCALE: hipLaunchKernelGGL(g_unscale, grid, blk, 0, s, probs, items); break;
    case G_INIT_STATE: hipLaunchKernelGGL(g_init_state, grid, dim3(64), 0, s, probs, items); break;
    case G_GATHER: hipLaunchKernelGGL(g_gather, grid, dim3(64), 0, s, probs, items); break;
    default: break;
  }
}

}  // namespace pogs
