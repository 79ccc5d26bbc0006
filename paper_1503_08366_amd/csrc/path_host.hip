// pogs_solve_path: R problems on one context's matrix, iterated together with
// stacked right-hand sides (matrix products on MFMA) until every problem has
// stopped.  Host side: packing the per-problem functions column-interleaved,
// state allocation, graph-captured iteration chunks, results.
#include <chrono>
#include <cstdio>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "ctx.hpp"
#include "hostutil.hpp"
#include "path.hpp"
#include "upload.hpp"

using namespace pogs;

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Per-problem functions packed as [len][Rp] (problem index fastest), float64
// a, b, c, d, e planes (prm) and the h codes (h), read straight from the
// callers' descriptors (stride 0 or 1) and validated on the way with the
// checks of expand_fn; columns r >= R are zero.  Element ranges run on the
// host pool's threads, writes contiguous over the problems.
int pack_fns(const pogs_fn *fs, int R, int len, int Rp, std::unique_ptr<double[]> *prm,
             std::unique_ptr<uint8_t[]> *h) {
  for (int r = 0; r < R; ++r)
    if (fs[r].len != len || !fs[r].h || (fs[r].stride != 0 && fs[r].stride != 1)) return POGS_EINVAL;
  const size_t tot = (size_t)len * Rp;
  prm->reset(new (std::nothrow) double[5 * tot]);
  h->reset(new (std::nothrow) uint8_t[tot]);
  if (!*prm || !*h) return POGS_ENOMEM;
  double *P = prm->get();
  uint8_t *H = h->get();
  std::atomic<int> bad{0};
  const int parts = len >= 4096 ? 16 : 1;
  auto body = [&](int part) {
    const int i0 = (int)((int64_t)len * part / parts), i1 = (int)((int64_t)len * (part + 1) / parts);
    bool ok = true;
    for (int i = i0; i < i1; ++i) {
      const size_t e0 = (size_t)i * Rp;
      for (int r = 0; r < R; ++r) {
        const pogs_fn &F = fs[r];
        const int64_t k = F.stride ? i : 0;
        const uint8_t hc = F.h[k];
        const double a = F.a ? F.a[k] : 1.0, b = F.b ? F.b[k] : 0.0, c = F.c ? F.c[k] : 1.0;
        const double d = F.d ? F.d[k] : 0.0, e = F.e ? F.e[k] : 0.0;
        ok = ok && fn_entry_ok(hc, a, b, c, d, e);
        P[e0 + r] = a;
        P[tot + e0 + r] = b;
        P[2 * tot + e0 + r] = c;
        P[3 * tot + e0 + r] = d;
        P[4 * tot + e0 + r] = e;
        H[e0 + r] = hc;
      }
      for (int r = R; r < Rp; ++r) {
        for (int q = 0; q < 5; ++q) P[q * tot + e0 + r] = 0.0;
        H[e0 + r] = 0;
      }
    }
    if (!ok) bad.store(1, std::memory_order_relaxed);
  };
  if (parts > 1) host_pool().run(parts, body);
  else body(0);
  return bad.load(std::memory_order_relaxed) ? POGS_EINVAL : POGS_OK;
}

}  // namespace

extern "C" int pogs_solve_path(pogs_ctx *ctx, int32_t R, const pogs_fn *f, const pogs_fn *g, const pogs_params *params,
                               pogs_result *out) {
  if (!ctx || !f || !g || !out || R < 1 || R > 256) return POGS_EINVAL;
  if (ctx->dt != POGS_F32 || ctx->m < ctx->n) return POGS_EUNSUPPORTED;
  pogs_params prm = params ? *params : ctx->params;
  if (check_params(prm)) return POGS_EINVAL;
  if (ctx->proj != POGS_PROJ_DIRECT || prm.projection != POGS_PROJ_DIRECT || prm.stop_rule != POGS_STOP_RESIDUAL)
    return POGS_EUNSUPPORTED;
  const double t0 = now_ms();
  const int m = (int)ctx->m, n = (int)ctx->n;
  int rc;
  for (int r = 0; r < R; ++r)
    if (out[r].mem != POGS_HOST && out[r].mem != POGS_DEVICE) return POGS_EINVAL;
  hipStream_t s = ctx->stream;
  const int Rp = (int)round_up(R, 64);
  std::unique_ptr<double[]> fprm, gprm;
  std::unique_ptr<uint8_t[]> fhh, ghh;
  const double t_expand = now_ms();
  if ((rc = pack_fns(f, R, m, Rp, &fprm, &fhh)) || (rc = pack_fns(g, R, n, Rp, &gprm, &ghh))) return rc;
  const double t_pack = now_ms();

  PathArgs p{};
  p.m = m;
  p.n = n;
  p.ld = ctx->ld;
  p.q = ctx->q;
  p.ldk = ctx->ldk;
  p.R = R;
  p.Rp = Rp;
  p.rows_per_block = 8;  // many small blocks: the split-K sums run in parallel
  p.nbx = (int)cdiv(n, p.rows_per_block);
  p.nby = (int)cdiv(m, p.rows_per_block);
  p.nb_pri = p.nby;
  p.nb_dual = p.nbx;
  p.alpha = (float)prm.alpha;
  p.delta = prm.delta;
  p.tau = prm.tau;
  p.eps_abs = prm.eps_abs;
  p.eps_rel = prm.eps_rel;
  p.max_iter = prm.max_iter;
  p.adaptive = prm.adaptive_rho ? 1 : 0;
  p.A = (const float *)ctx->A;
  p.Kinv = (const float *)ctx->Kinv;

  DevArena tmp(s);
  const size_t tf = (size_t)m * Rp, tg = (size_t)n * Rp;
  double *f0, *g0;
  uint8_t *fh0, *gh0, *fh, *gh;
  float *fs, *gs, *state, *part, *outs;
  double *slots, *percol, *obj;
  int *ints;
  const size_t state_floats = 2 * tg + 3 * tg + 2 * tf + 3 * tf + tg;
  const size_t nslots = (size_t)(p.nbx + p.nby + p.nb_pri + p.nb_dual) * Rp;
  if ((rc = tmp.alloc((void **)&f0, 5 * tf * 8)) || (rc = tmp.alloc((void **)&g0, 5 * tg * 8)) ||
      (rc = tmp.alloc((void **)&fh0, tf)) || (rc = tmp.alloc((void **)&gh0, tg)) || (rc = tmp.alloc((void **)&fh, tf)) ||
      (rc = tmp.alloc((void **)&gh, tg)) || (rc = tmp.alloc((void **)&fs, 5 * tf * 4)) ||
      (rc = tmp.alloc((void **)&gs, 5 * tg * 4)) || (rc = tmp.alloc((void **)&state, state_floats * 4)) ||
      (rc = tmp.alloc((void **)&part, path_part_floats(m, n, Rp) * 4)) ||
      (rc = tmp.alloc((void **)&outs, (size_t)R * 2 * (m + n) * 4)) || (rc = tmp.alloc((void **)&slots, nslots * 8)) ||
      (rc = tmp.alloc((void **)&percol, (size_t)6 * Rp * 8)) || (rc = tmp.alloc((void **)&obj, (size_t)Rp * 8)) ||
      (rc = tmp.alloc((void **)&ints, (size_t)(5 * Rp + 64) * 4)))
    return rc;
  POGS_HIP_TRY(hipMemcpyAsync(f0, fprm.get(), 5 * tf * 8, hipMemcpyHostToDevice, s));
  POGS_HIP_TRY(hipMemcpyAsync(g0, gprm.get(), 5 * tg * 8, hipMemcpyHostToDevice, s));
  POGS_HIP_TRY(hipMemcpyAsync(fh0, fhh.get(), tf, hipMemcpyHostToDevice, s));
  POGS_HIP_TRY(hipMemcpyAsync(gh0, ghh.get(), tg, hipMemcpyHostToDevice, s));
  launch_path_scale_fn(f0, fh0, m, Rp, ctx->D, true, fh, fs, fs + tf, fs + 2 * tf, fs + 3 * tf, fs + 4 * tf, s);
  launch_path_scale_fn(g0, gh0, n, Rp, ctx->E, false, gh, gs, gs + tg, gs + 2 * tg, gs + 3 * tg, gs + 4 * tg, s);
  p.fh = fh;
  p.gh = gh;
  p.fa = fs;
  p.fb = fs + tf;
  p.fc = fs + 2 * tf;
  p.fd = fs + 3 * tf;
  p.fe = fs + 4 * tf;
  p.ga = gs;
  p.gb = gs + tg;
  p.gc = gs + 2 * tg;
  p.gd = gs + 3 * tg;
  p.ge = gs + 4 * tg;
  float *sp = state;
  p.XX = sp; sp += 2 * tg;
  p.Xt = sp; sp += tg;
  p.Mu = sp; sp += tg;
  p.Cx = sp; sp += tg;
  p.DN = sp; sp += 2 * tf;
  p.Y = sp; sp += tf;
  p.Yt = sp; sp += tf;
  p.Yh = sp; sp += tf;
  p.Rhs = sp; sp += tg;
  POGS_HIP_TRY(hipMemsetAsync(state, 0, state_floats * 4, s));
  p.s_mu = slots;
  p.s_yh = p.s_mu + (size_t)p.nbx * Rp;
  p.s_pri = p.s_yh + (size_t)p.nby * Rp;
  p.s_dual = p.s_pri + (size_t)p.nb_pri * Rp;
  p.rho = percol;
  p.rescale = percol + Rp;
  p.r_pri = percol + 2 * Rp;
  p.r_dual = percol + 3 * Rp;
  p.eps_pri = percol + 4 * Rp;
  p.eps_dual = percol + 5 * Rp;
  p.l = ints;
  p.u = ints + Rp;
  p.iters = ints + 2 * Rp;
  p.done = ints + 3 * Rp;
  p.status = ints + 4 * Rp;
  p.all_done = ints + 5 * Rp;
  {
    std::vector<double> hc(6 * (size_t)Rp, 0.0);
    for (int r = 0; r < Rp; ++r) {
      hc[r] = prm.rho0;
      hc[Rp + r] = 1.0;
    }
    std::vector<int> hi(5 * (size_t)Rp + 64, 0);
    for (int r = 0; r < Rp; ++r) hi[4 * Rp + r] = -1;
    POGS_HIP_TRY(hipMemcpyAsync(percol, hc.data(), hc.size() * 8, hipMemcpyHostToDevice, s));
    POGS_HIP_TRY(hipMemcpyAsync(ints, hi.data(), hi.size() * 4, hipMemcpyHostToDevice, s));
    POGS_HIP_TRY(hipStreamSynchronize(s));
  }
  // iterate in captured chunks until every problem has stopped
  const double t_upload = now_ms();
  const int chunk = std::max(1, prm.chunk_iters > 0 ? prm.chunk_iters : 20);
  hipGraph_t graph;
  hipGraphExec_t exec;
  POGS_HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  for (int i = 0; i < chunk; ++i) launch_path_iteration(p, part, s);
  POGS_HIP_TRY(hipStreamEndCapture(s, &graph));
  if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return POGS_EDEVICE;
  }
  (void)hipGraphDestroy(graph);
  const double t_capture = now_ms();
  int all_done = 0;
  int guard = 0;
  const int max_launches = (int)cdiv(prm.max_iter, chunk) + 1;
  while (!all_done && guard++ < max_launches) {
    if (hipGraphLaunch(exec, s) != hipSuccess) break;
    if (hipMemcpyAsync(&all_done, p.all_done, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess) break;
    if (hipStreamSynchronize(s) != hipSuccess) break;
  }
  const double t_iter = now_ms();
  (void)hipGraphExecDestroy(exec);
  POGS_HIP_TRY(hipGetLastError());
  const double t_destroy = now_ms();
  launch_path_unscale(p, ctx->D, ctx->E, f0, fh0, g0, gh0, outs, obj, s);
  std::vector<double> hc(6 * (size_t)Rp), hobj(Rp);
  std::vector<int> hi(5 * (size_t)Rp);
  POGS_HIP_TRY(hipMemcpyAsync(hc.data(), percol, hc.size() * 8, hipMemcpyDeviceToHost, s));
  POGS_HIP_TRY(hipMemcpyAsync(hi.data(), ints, hi.size() * 4, hipMemcpyDeviceToHost, s));
  POGS_HIP_TRY(hipMemcpyAsync(hobj.data(), obj, (size_t)Rp * 8, hipMemcpyDeviceToHost, s));
  // host outputs: the R result blocks in one copy to pinned memory, then
  // scattered on the host; device outputs: copies on the device
  const size_t blk = 2 * (size_t)(m + n);
  bool any_host = false;
  for (int r = 0; r < R; ++r) any_host |= out[r].mem == POGS_HOST;
  float *staged = nullptr;
  if (any_host) {
    staged = (float *)pinned_stage().acquire((size_t)R * blk * 4);
    if (!staged) return POGS_ENOMEM;
    const hipError_t e = hipMemcpyAsync(staged, outs, (size_t)R * blk * 4, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) {
      pinned_stage().release(s);
      return POGS_EDEVICE;
    }
  }
  for (int r = 0; r < R; ++r) {
    if (out[r].mem != POGS_DEVICE) continue;
    const float *o = outs + (size_t)r * blk;
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    if (out[r].x) POGS_HIP_TRY(hipMemcpyAsync(out[r].x, o, (size_t)n * 4, k, s));
    if (out[r].y) POGS_HIP_TRY(hipMemcpyAsync(out[r].y, o + n, (size_t)m * 4, k, s));
    if (out[r].mu) POGS_HIP_TRY(hipMemcpyAsync(out[r].mu, o + n + m, (size_t)n * 4, k, s));
    if (out[r].nu) POGS_HIP_TRY(hipMemcpyAsync(out[r].nu, o + 2 * n + m, (size_t)m * 4, k, s));
  }
  const hipError_t se = hipStreamSynchronize(s);
  if (any_host) {
    if (se == hipSuccess)
      for (int r = 0; r < R; ++r) {
        if (out[r].mem != POGS_HOST) continue;
        const float *o = staged + (size_t)r * blk;
        if (out[r].x) std::memcpy(out[r].x, o, (size_t)n * 4);
        if (out[r].y) std::memcpy(out[r].y, o + n, (size_t)m * 4);
        if (out[r].mu) std::memcpy(out[r].mu, o + n + m, (size_t)n * 4);
        if (out[r].nu) std::memcpy(out[r].nu, o + 2 * n + m, (size_t)m * 4);
      }
    pinned_stage().release(s);
  }
  POGS_HIP_TRY(se);
  POGS_HIP_TRY(hipGetLastError());
  const double ms = now_ms() - t0;
  if (prm.verbose)
    fprintf(stderr,
            "pogs path: %d problems: checks %.1f ms, pack %.1f ms, upload and scale %.1f ms, capture %.1f ms, "
            "iterations %.1f ms, graph destroy %.1f ms, results %.1f ms\n",
            R, t_expand - t0, t_pack - t_expand, t_upload - t_pack, t_capture - t_upload, t_iter - t_capture,
            t_destroy - t_iter, now_ms() - t_destroy);
  for (int r = 0; r < R; ++r) {
    out[r].optval = hobj[r];
    out[r].rho = hc[r];
    out[r].r_pri = hc[2 * Rp + r];
    out[r].r_dual = hc[3 * Rp + r];
    out[r].eps_pri = hc[4 * Rp + r];
    out[r].eps_dual = hc[5 * Rp + r];
    out[r].iters = hi[2 * Rp + r];
    out[r].status = hi[4 * Rp + r] < 0 ? POGS_MAXITER : hi[4 * Rp + r];
    out[r].ms_setup = ctx->ms_setup;
    out[r].ms_solve = ms;
    out[r].cg_steps = 0;
    out[r].gap = NAN;
    out[r].eps_gap = NAN;
  }
  return POGS_OK;
}
