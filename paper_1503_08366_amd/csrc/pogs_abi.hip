// C ABI of the graph-form ADMM library (see include/pogs.h): argument checks,
// context and device-memory management, the setup pipeline, and the host loop
// that replays captured iteration chunks until the device stop flag is set.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "internal.hpp"
#include "prox.hpp"
#include "hostutil.hpp"
#include "ctx.hpp"
#include "upload.hpp"

using namespace pogs;

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

extern "C" {

const char *pogs_strerror(int code) {
  switch (code) {
    case POGS_OK: return "ok";
    case POGS_EINVAL: return "invalid argument";
    case POGS_ENOMEM: return "out of memory";
    case POGS_EDEVICE: return "HIP runtime error";
    case POGS_EAGAIN: return "request does not fit the memory budget or the queue is full";
    case POGS_ENOTFOUND: return "unknown ticket";
    case POGS_EUNSUPPORTED: return "not supported by the library";
    case POGS_ETOOBIG: return "input exceeds the fixed device buffer of an allocation-free entry point";
    default: return "unknown error";
  }
}

int pogs_params_default(pogs_params *p) {
  if (!p) return POGS_EINVAL;
  p->eps_abs = 1e-4;
  p->eps_rel = 1e-3;
  p->max_iter = 10000;
  p->rho0 = 1.0;
  p->alpha = 1.7;
  p->delta = 1.05;
  p->tau = 0.8;
  p->adaptive_rho = 1;
  p->equil_iters = 10;
  p->eps_cmp = 0.0;
  p->chunk_iters = 20;
  p->verbose = 0;
  p->projection = POGS_PROJ_DIRECT;
  p->cg_max_iter = 10;
  p->cg_tol = 0.1;
  p->stop_rule = POGS_STOP_RESIDUAL;
  p->autotune = 1;
  p->sparse_segment = 0;
  return POGS_OK;
}

}  // extern "C"

namespace {
// The library's stream for the calling thread on the current device (a
// NULL stream argument): created on first use and kept until the process
// ends, so a context neither creates nor destroys a stream (destroying one
// cost pogs_free about 140 us, measured on MI355X).  Calls are synchronous,
// so the contexts of one thread can share it.
hipStream_t library_stream() {
  static thread_local std::vector<std::pair<int, hipStream_t>> streams;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  for (auto &e : streams)
    if (e.first == dev) return e.second;
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
  streams.push_back({dev, st});
  return st;
}
}  // namespace

extern "C" {

int pogs_free(pogs_ctx *ctx) {
  if (!ctx) return POGS_OK;
  // drained, the context's blocks can be kept for the next context
  const bool idle = !ctx->stream || hipStreamSynchronize(ctx->stream) == hipSuccess;
  ctx->arena.free_all(idle);
  delete ctx;
  return POGS_OK;
}

}  // extern "C"

namespace {

template <typename T> int init_impl(pogs_ctx *c, const void *A, pogs_dtype sdt, pogs_order ord, int64_t lda,
                                    pogs_mem mem) {
  const int m = (int)c->m, n = (int)c->n;
  hipStream_t s = c->stream;
  DevArena tmp(s);
  int rc;
  // -- layout -------------------------------------------------------------
  if ((rc = c->arena.alloc(&c->A, (size_t)m * c->ld * sizeof(T)))) return rc;
  const size_t selem = sdt == POGS_F32 ? 4 : 8;
  const size_t src_elems = ord == POGS_ROW_MAJOR ? (size_t)(m - 1) * lda + n : (size_t)(n - 1) * lda + m;
  const void *src = A;
  if (mem == POGS_HOST) {
    void *stage;
    if ((rc = tmp.alloc(&stage, src_elems * selem))) return rc;
    POGS_HIP_TRY(host_uploader().upload(stage, A, src_elems * selem, s));
    src = stage;
  }
  unsigned *flags;  // [0] non-finite A, [1] factorisation failures, [2] factor step flag
  if ((rc = tmp.alloc((void **)&flags, 64))) return rc;
  POGS_HIP_TRY(hipMemsetAsync(flags, 0, 64, s));
  launch_layout<T>(src, sdt, ord, lda, m, n, (T *)c->A, c->ld, flags, s);
  // -- equilibration ------------------------------------------------------
  if ((rc = c->arena.alloc((void **)&c->D, (size_t)m * 8))) return rc;
  if ((rc = c->arena.alloc((void **)&c->E, (size_t)n * 8))) return rc;
  unsigned *cnt;
  const size_t ncnt = (size_t)cdiv(n, 128) + 16;
  if ((rc = tmp.alloc((void **)&cnt, ncnt * sizeof(unsigned)))) return rc;
  POGS_HIP_TRY(hipMemsetAsync(cnt, 0, ncnt * sizeof(unsigned), s));
  {
    const size_t wsb = equil_workspace_bytes(m, n);
    double *ws;
    if ((rc = tmp.alloc((void **)&ws, wsb))) return rc;
    double eps = c->params.eps_cmp > 0.0 ? c->params.eps_cmp
                                         : (sizeof(T) == 4 ? (double)FLT_EPSILON : DBL_EPSILON);
    if ((rc = run_equilibrate<T>((T *)c->A, m, n, c->ld, c->params.equil_iters, eps, c->D, c->E, ws, wsb, cnt, s)))
      return rc;
  }
  // -- Gram and factorisation (direct projection) -------------------------
  if (c->proj == POGS_PROJ_CGLS) {
    POGS_HIP_TRY(hipMemcpyAsync(c->flags_host, flags, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    return POGS_OK;
  }
  const int Q = c->Q;
  double *K;
  if ((rc = tmp.alloc((void **)&K, (size_t)Q * Q * 8))) return rc;
  if ((rc = c->arena.alloc(&c->Kinv, (size_t)c->q * c->ldk * sizeof(T)))) return rc;
  {
    // one block serves the Gram partials, then the factor's workspace
    // (stream order separates the two uses)
    const size_t gb = gram_workspace_bytes(m, n, sizeof(T));
    const size_t fb = factor_workspace_bytes(Q);
    void *ws;
    if ((rc = tmp.alloc(&ws, std::max(gb, fb)))) return rc;
    if ((rc = run_gram<T>((const T *)c->A, m, n, c->ld, K, Q, (float *)ws, (double *)ws, gb, s))) return rc;
    if ((rc = run_factor_inverse<T>(K, c->q, Q, (T *)c->Kinv, c->ldk, (double *)ws, flags + 1, s))) return rc;
  }
  // read back once pogs_init has queued the rest of its work (the frees of
  // the temporaries above go in stream order meanwhile)
  POGS_HIP_TRY(hipMemcpyAsync(c->flags_host, flags, 2 * sizeof(unsigned), hipMemcpyDeviceToHost, s));
  return POGS_OK;
}

template <typename T> int alloc_iteration(pogs_ctx *c) {
  static_assert(sizeof(Ctrl) <= PinnedSlab::kChunk, "control block larger than a pinned slab chunk");
  const int m = (int)c->m, n = (int)c->n;
  // gemv_t geometry over the n columns (same for both orientations); a sparse
  // context's residual sums come from its row passes over A^ and A^T
  gemv_t_geometry(m, n, sizeof(T), &c->splits, &c->rps, &c->ncolp);
  c->nbx = (int)cdiv(n, kBlock);
  c->nby = (int)cdiv(m, kBlock);
  c->n_pri = c->sparse ? c->sp_grid : gemv_n_blocks(m, n, sizeof(T), 0);
  c->n_dual = c->sparse ? c->sp_gridt : (int)cdiv(n, kFinishCols);
  if (c->sparse) c->splits = 1;  // no column-sum partials
  // prox sums (two parities), residual sums, CGLS sums (||s||^2 and s^T p by
  // step parity, ||q||^2), then the unscale kernel's sums
  c->fp_blocks = one_pass_blocks(m, n, c->ld, (int)sizeof(T), c->sparse);
  c->smu_cap = std::max(c->nbx, c->n_dual);
  c->syh_cap = std::max({c->nby, c->splits, c->fp_blocks});
  c->fused = false;
  const int nslots = 2 * (c->smu_cap + c->syh_cap) + std::max(c->n_pri, c->fp_blocks) + c->n_dual +
                     4 * c->n_dual + c->n_pri + 2 * (c->nbx + c->nby) + c->nbx + c->nby;
  const int ntiles = (int)cdiv(n, gemv_t_tile(sizeof(T)));
  // raw functions: fh0 | gh0 | f0 | g0, uploaded in one copy
  Carve raw;
  raw.take(m);
  c->off_gh0 = raw.take(n);
  c->off_f0 = raw.take((size_t)5 * m * 8);
  c->off_g0 = raw.take((size_t)5 * n * 8);
  c->fn_bytes = raw.off;
  // every per-context iteration buffer in one allocation
  Carve cv;
  const size_t o_vec = cv.take(c->vec_elems() * sizeof(T));
  const size_t o_fh = cv.take(m), o_gh = cv.take(n);
  const size_t o_fs = cv.take((size_t)5 * m * sizeof(T)), o_gs = cv.take((size_t)5 * n * sizeof(T));
  const size_t o_raw = cv.take(c->fn_bytes);
  const size_t o_part = cv.take((size_t)std::max(c->splits, c->fp_blocks) * 2 * c->ncolp * 8);
  const size_t o_slots = cv.take((size_t)nslots * 8);
  const size_t o_cnt = cv.take((size_t)(ntiles + 64) * sizeof(unsigned));
  const size_t o_ctrl = cv.take(sizeof(Ctrl));
  const size_t o_obj = cv.take(64);
  char *base;
  int rc;
  if ((rc = c->arena.alloc((void **)&base, cv.off))) return rc;
  c->vec = base + o_vec;
  c->fh = (uint8_t *)(base + o_fh);
  c->gh = (uint8_t *)(base + o_gh);
  c->fs = base + o_fs;
  c->gs = base + o_gs;
  c->fn_raw = base + o_raw;
  c->fh0 = (uint8_t *)c->fn_raw;
  c->gh0 = (uint8_t *)c->fn_raw + c->off_gh0;
  c->f0 = (double *)((char *)c->fn_raw + c->off_f0);
  c->g0 = (double *)((char *)c->fn_raw + c->off_g0);
  c->part = (double *)(base + o_part);
  c->slots = (double *)(base + o_slots);
  c->counters = (unsigned *)(base + o_cnt);
  c->ctrl = (Ctrl *)(base + o_ctrl);
  c->obj_dev = (double *)(base + o_obj);
  POGS_HIP_TRY(hipMemsetAsync(c->vec, 0, c->vec_elems() * sizeof(T), c->stream));
  POGS_HIP_TRY(hipMemsetAsync(c->counters, 0, (size_t)(ntiles + 64) * sizeof(unsigned), c->stream));
  c->ctrl_host = (Ctrl *)pinned_slab().get();
  c->obj_host = (double *)pinned_slab().get();
  if (!c->ctrl_host || !c->obj_host) return POGS_ENOMEM;
  return POGS_OK;
}

// Load policy of the passes over A.  Default: stream (non-temporal loads) a
// matrix larger than kStreamMatrixBytes.  With params.autotune the four
// policies (row passes x column passes, cached or streamed) are timed on the
// context: after one warm projection, four projections (pass 1, the solve with
// K^-1, pass 2) each, in sequence so that what one pass leaves in the caches
// for the next counts, with HIP events on the context's stream; the fastest is
// kept, per (m, n, dtype) for the process.  The policy changes no arithmetic.
struct TuneKey {
  int64_t m, n;
  int dt;
  bool operator<(const TuneKey &o) const {
    return m != o.m ? m < o.m : n != o.n ? n < o.n : dt < o.dt;
  }
};
std::mutex &tune_mutex() {
  static std::mutex mu;
  return mu;
}
std::map<TuneKey, std::pair<int, int>> &tune_table() {
  static std::map<TuneKey, std::pair<int, int>> t;
  return t;
}

template <typename T> int tune_loads(pogs_ctx *c) {
  const int big = (size_t)c->m * c->ld * sizeof(T) > kStreamMatrixBytes ? 1 : 0;
  c->nt_rows = c->nt_cols = big;
  if (!c->params.autotune) return POGS_OK;
  const TuneKey key{c->m, c->n, (int)c->dt};
  {
    std::lock_guard<std::mutex> g(tune_mutex());
    auto it = tune_table().find(key);
    if (it != tune_table().end()) {
      c->nt_rows = it->second.first;
      c->nt_cols = it->second.second;
      return POGS_OK;
    }
  }
  hipStream_t s = c->stream;
  POGS_HIP_TRY(hipMemsetAsync(c->ctrl, 0, sizeof(Ctrl), s));  // no stop flag: every pass runs
  hipEvent_t e0, e1;
  POGS_HIP_TRY(hipEventCreate(&e0));
  POGS_HIP_TRY(hipEventCreate(&e1));
  // the four candidates interleaved over several rounds, each keeping its
  // best time (noise then hits them alike); the size rule's policy is left
  // only for one at least 2 % faster (the candidates are often within noise)
  float best_ms[4] = {1e30f, 1e30f, 1e30f, 1e30f};
  const bool solve = c->Kinv != nullptr;  // the solve only where the factor exists (a CGLS context has none)
  for (int round = 0; round < 4; ++round)
    for (int cand = 0; cand < 4; ++cand) {
      IterArgs<T> p = c->iter_args<T>();
      p.nt_rows = cand & 1;
      p.nt_cols = cand >> 1;
      for (int w = 1; w < 4; ++w)
        if (w != 2 || solve) launch_iteration_part<T>(p, w, c->splits, c->rps, c->ncolp, s);
      POGS_HIP_TRY(hipEventRecord(e0, s));
      for (int r = 0; r < 2; ++r)
        for (int w = 1; w < 4; ++w)
          if (w != 2 || solve) launch_iteration_part<T>(p, w, c->splits, c->rps, c->ncolp, s);
      POGS_HIP_TRY(hipEventRecord(e1, s));
      POGS_HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      POGS_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      best_ms[cand] = std::min(best_ms[cand], ms);
    }
  const int def = big | (big << 1);
  int pick = def;
  for (int cand = 0; cand < 4; ++cand)
    if (best_ms[cand] < best_ms[pick] && best_ms[cand] < 0.98f * best_ms[def]) pick = cand;
  const int best_r = pick & 1, best_c = pick >> 1;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  POGS_HIP_TRY(hipGetLastError());
  c->nt_rows = best_r;
  c->nt_cols = best_c;
  std::lock_guard<std::mutex> g(tune_mutex());
  tune_table()[key] = {best_r, best_c};
  return POGS_OK;
}

}  // namespace

extern "C" int pogs_init(pogs_ctx **out, int64_t m, int64_t n, const void *A, pogs_dtype dt, pogs_order ord,
                         int64_t lda, pogs_mem mem, const pogs_params *params, void *stream) {
  if (!out) return POGS_EINVAL;
  *out = nullptr;
  if (m <= 0 || n <= 0 || !A || m > (1LL << 31) - 1 || n > (1LL << 31) - 1) return POGS_EINVAL;
  if (dt != POGS_F32 && dt != POGS_F64) return POGS_EINVAL;
  if (ord != POGS_ROW_MAJOR && ord != POGS_COL_MAJOR) return POGS_EINVAL;
  if (mem != POGS_HOST && mem != POGS_DEVICE) return POGS_EINVAL;
  if (lda < (ord == POGS_ROW_MAJOR ? n : m)) return POGS_EINVAL;
  if ((size_t)round_up(m, 64) * (size_t)round_up(n, 64) > (size_t)(1ULL << 40)) return POGS_EINVAL;
  pogs_params p;
  pogs_params_default(&p);
  if (params) p = *params;
  if (check_params(p)) return POGS_EINVAL;
  // the factor of I + G would exceed 8 GiB
  if (p.projection == POGS_PROJ_DIRECT && std::min(m, n) > 32768) return POGS_EUNSUPPORTED;
  const double t0 = now_ms();
  pogs_ctx *c = new (std::nothrow) pogs_ctx();
  if (!c) return POGS_ENOMEM;
  c->m = m;
  c->n = n;
  c->dt = dt;
  c->params = p;
  c->proj = p.projection;
  c->ld = (int)round_up(n, 64);
  c->q = (int)std::min(m, n);
  c->Q = (int)round_up(c->q, 64);
  c->ldk = (int)round_up(c->q, 64);
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else if (!(c->stream = library_stream())) {
    delete c;
    return POGS_EDEVICE;
  }
  c->arena.stream = c->stream;
  // [0] non-finite A, [1] factorisation failures: read after the one wait below
  c->flags_host = (unsigned *)pinned_slab().get();
  int rc = c->flags_host ? POGS_OK : POGS_ENOMEM;
  if (!rc) {
    c->flags_host[0] = c->flags_host[1] = 0;
    rc = dt == POGS_F32 ? init_impl<float>(c, A, dt, ord, lda, mem) : init_impl<double>(c, A, dt, ord, lda, mem);
  }
  if (!rc) rc = dt == POGS_F32 ? alloc_iteration<float>(c) : alloc_iteration<double>(c);
  if (!rc) rc = dt == POGS_F32 ? tune_loads<float>(c) : tune_loads<double>(c);
  if (hipStreamSynchronize(c->stream) != hipSuccess && !rc) rc = POGS_EDEVICE;
  if (!rc && hipGetLastError() != hipSuccess) rc = POGS_EDEVICE;
  if (!rc && c->flags_host[0]) rc = POGS_EINVAL;   // non-finite entries in A
  if (!rc && c->flags_host[1]) rc = POGS_EDEVICE;  // I + G not positive definite numerically
  if (rc) {
    delete c;
    return rc;
  }
  c->ms_setup = now_ms() - t0;
  *out = c;
  return POGS_OK;
}

namespace {

// Host copy of a CSR input checked entry by entry (values widened to double).
struct HostCsr {
  std::vector<int> rp, ci;
  std::vector<double> va;
};

int read_csr(int64_t m, int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *colind, const void *val,
             pogs_dtype dt, pogs_mem mem, HostCsr *h) {
  std::vector<int64_t> rp((size_t)m + 1);
  std::vector<int32_t> ci((size_t)nnz);
  const size_t es = dt == POGS_F32 ? 4 : 8;
  std::vector<char> raw((size_t)nnz * es);
  if (mem == POGS_DEVICE) {
    if (hipMemcpy(rp.data(), rowptr, rp.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) return POGS_EDEVICE;
    if (nnz && hipMemcpy(ci.data(), colind, ci.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) return POGS_EDEVICE;
    if (nnz && hipMemcpy(raw.data(), val, raw.size(), hipMemcpyDeviceToHost) != hipSuccess) return POGS_EDEVICE;
  } else {
    std::memcpy(rp.data(), rowptr, rp.size() * 8);
    if (nnz) std::memcpy(ci.data(), colind, ci.size() * 4);
    if (nnz) std::memcpy(raw.data(), val, raw.size());
  }
  if (rp[0] != 0 || rp[(size_t)m] != nnz) return POGS_EINVAL;
  for (int64_t i = 0; i < m; ++i)
    if (rp[(size_t)i + 1] < rp[(size_t)i]) return POGS_EINVAL;
  h->rp.resize((size_t)m + 1);
  for (int64_t i = 0; i <= m; ++i) h->rp[(size_t)i] = (int)rp[(size_t)i];
  h->ci.assign(ci.begin(), ci.end());
  h->va.resize((size_t)nnz);
  for (int64_t k = 0; k < nnz; ++k) {
    if (ci[(size_t)k] < 0 || ci[(size_t)k] >= n) return POGS_EINVAL;
    const double v = dt == POGS_F32 ? (double)((const float *)raw.data())[k] : ((const double *)raw.data())[k];
    if (!std::isfinite(v)) return POGS_EINVAL;
    h->va[(size_t)k] = v;
  }
  return POGS_OK;
}

// A^T in compressed rows split into column segments of seg columns (rows of
// A): the entries of row j of A^T whose column i lies in segment s = i / seg
// form row piece s n + j, stored in that order.  A counting sort over the
// pieces that keeps the row order of A inside each piece (deterministic).
void transpose_csr(const HostCsr &a, int n, int seg, HostCsr *t) {
  const size_t nnz = a.ci.size();
  const int m = (int)a.rp.size() - 1;
  const size_t pieces = (size_t)cdiv(m, seg) * n;
  t->rp.assign(pieces + 1, 0);
  for (int i = 0; i < m; ++i) {
    const size_t base = (size_t)(i / seg) * n;
    for (int k = a.rp[(size_t)i]; k < a.rp[(size_t)i + 1]; ++k) ++t->rp[base + a.ci[(size_t)k] + 1];
  }
  for (size_t b = 0; b < pieces; ++b) t->rp[b + 1] += t->rp[b];
  std::vector<int> cur(t->rp.begin(), t->rp.end() - 1);
  t->ci.resize(nnz);
  t->va.resize(nnz);
  for (int i = 0; i < m; ++i) {
    const size_t base = (size_t)(i / seg) * n;
    for (int k = a.rp[(size_t)i]; k < a.rp[(size_t)i + 1]; ++k) {
      const int pos = cur[base + a.ci[(size_t)k]]++;
      t->ci[(size_t)pos] = i;
      t->va[(size_t)pos] = a.va[(size_t)k];
    }
  }
}

template <typename T> int init_sparse_impl(pogs_ctx *c, const HostCsr &a, const HostCsr &t) {
  const int m = (int)c->m, n = (int)c->n;
  const size_t nnz = a.ci.size();
  hipStream_t s = c->stream;
  int rc;
  sparse_shape(m, (int64_t)nnz, &c->sp_lpr, &c->sp_grid);
  sparse_seg_shape(n, c->sp_nseg, (int64_t)nnz, &c->sp_lprt, &c->sp_gridt);
  if ((rc = c->arena.alloc((void **)&c->sp_rp, ((size_t)m + 1) * 4))) return rc;
  if ((rc = c->arena.alloc((void **)&c->sp_rpt, t.rp.size() * 4))) return rc;
  if ((rc = c->arena.alloc((void **)&c->sp_ci, std::max<size_t>(nnz, 1) * 4))) return rc;
  if ((rc = c->arena.alloc((void **)&c->sp_cit, std::max<size_t>(nnz, 1) * 4))) return rc;
  if ((rc = c->arena.alloc(&c->sp_va, std::max<size_t>(nnz, 1) * sizeof(T)))) return rc;
  if ((rc = c->arena.alloc(&c->sp_vat, std::max<size_t>(nnz, 1) * sizeof(T)))) return rc;
  if ((rc = c->arena.alloc(&c->sp_pair, (size_t)2 * m * sizeof(T)))) return rc;
  std::vector<T> va(a.va.begin(), a.va.end()), vat(t.va.begin(), t.va.end());
  HostUploader &up = host_uploader();
  POGS_HIP_TRY(up.upload(c->sp_rp, a.rp.data(), a.rp.size() * 4, s));
  POGS_HIP_TRY(up.upload(c->sp_rpt, t.rp.data(), t.rp.size() * 4, s));
  if (nnz) {
    POGS_HIP_TRY(up.upload(c->sp_ci, a.ci.data(), nnz * 4, s));
    POGS_HIP_TRY(up.upload(c->sp_cit, t.ci.data(), nnz * 4, s));
    POGS_HIP_TRY(up.upload(c->sp_va, va.data(), nnz * sizeof(T), s));
    POGS_HIP_TRY(up.upload(c->sp_vat, vat.data(), nnz * sizeof(T), s));
  }
  if ((rc = c->arena.alloc((void **)&c->D, (size_t)m * 8))) return rc;
  if ((rc = c->arena.alloc((void **)&c->E, (size_t)n * 8))) return rc;
  DevArena tmp(s);
  double *ws;
  if ((rc = tmp.alloc((void **)&ws, (2 * ((size_t)m + n) + 1024) * 8))) return rc;
  const double eps = c->params.eps_cmp > 0.0 ? c->params.eps_cmp : (sizeof(T) == 4 ? (double)FLT_EPSILON : DBL_EPSILON);
  const IterArgs<T> ia = c->iter_args<T>();
  run_equilibrate_sparse<T>(ia.sa, ia.sat, m, n, c->params.equil_iters, eps, c->D, c->E, ws, s);
  POGS_HIP_TRY(hipStreamSynchronize(s));  // the host copies above are pageable
  POGS_HIP_TRY(hipGetLastError());
  return POGS_OK;
}

}  // namespace

extern "C" int pogs_init_sparse(pogs_ctx **out, int64_t m, int64_t n, int64_t nnz, const int64_t *rowptr,
                                const int32_t *colind, const void *val, pogs_dtype dt, pogs_mem mem,
                                const pogs_params *params, void *stream) {
  if (!out) return POGS_EINVAL;
  *out = nullptr;
  if (m <= 0 || n <= 0 || nnz < 0 || !rowptr || (nnz > 0 && (!colind || !val))) return POGS_EINVAL;
  if (m > (1LL << 31) - 2 || n > (1LL << 31) - 2 || nnz > (1LL << 31) - 1) return POGS_EINVAL;
  if ((dt != POGS_F32 && dt != POGS_F64) || (mem != POGS_HOST && mem != POGS_DEVICE)) return POGS_EINVAL;
  pogs_params p;
  pogs_params_default(&p);
  if (params) p = *params;
  p.projection = POGS_PROJ_CGLS;
  if (check_params(p)) return POGS_EINVAL;
  const double t0 = now_ms();
  HostCsr a, t;
  int rc = read_csr(m, n, nnz, rowptr, colind, val, dt, mem, &a);
  if (rc) return rc;
  const int seg = p.sparse_segment > 0 ? (int)std::min<int64_t>(p.sparse_segment, m)
                                       : sparse_segment((int)m, (int)n, nnz, dt == POGS_F32 ? 4 : 8);
  transpose_csr(a, (int)n, seg, &t);
  pogs_ctx *c = new (std::nothrow) pogs_ctx();
  if (!c) return POGS_ENOMEM;
  c->m = m;
  c->n = n;
  c->dt = dt;
  c->params = p;
  c->proj = POGS_PROJ_CGLS;
  c->sparse = true;
  c->nnz = nnz;
  c->sp_nseg = (int)cdiv(m, (int64_t)seg);
  c->ld = (int)round_up(n, 64);
  c->q = (int)std::min(m, n);
  c->Q = (int)round_up(c->q, 64);
  c->ldk = c->Q;
  if (stream) {
    c->stream = (hipStream_t)stream;
  } else if (!(c->stream = library_stream())) {
    delete c;
    return POGS_EDEVICE;
  }
  c->arena.stream = c->stream;
  rc = dt == POGS_F32 ? init_sparse_impl<float>(c, a, t) : init_sparse_impl<double>(c, a, t);
  if (!rc) rc = dt == POGS_F32 ? alloc_iteration<float>(c) : alloc_iteration<double>(c);
  if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = POGS_EDEVICE;
  if (rc) {
    delete c;
    return rc;
  }
  c->ms_setup = now_ms() - t0;
  *out = c;
  return POGS_OK;
}


namespace {

template <typename T> int upload_fns(pogs_ctx *c, const pogs_fn *f, const pogs_fn *g) {
  const int m = (int)c->m, n = (int)c->n;
  hipStream_t s = c->stream;
  // one pinned staging copy of fh0 | gh0 | f0 | g0, validated and expanded
  // straight into the stage
  char *st = (char *)pinned_stage().acquire(c->fn_bytes);
  if (!st) return POGS_ENOMEM;
  int rc = stage_fn(f, m, (uint8_t *)st, (double *)(st + c->off_f0));
  if (!rc) rc = stage_fn(g, n, (uint8_t *)st + c->off_gh0, (double *)(st + c->off_g0));
  if (rc) {
    pinned_stage().release(s);
    return rc;
  }
  const hipError_t e = hipMemcpyAsync(c->fn_raw, st, c->fn_bytes, hipMemcpyHostToDevice, s);
  pinned_stage().release(s);
  if (e != hipSuccess) return POGS_EDEVICE;
  T *fsp = (T *)c->fs, *gsp = (T *)c->gs;
  // f^(y) = f(y / D), g^(x) = g(E x)  (Section 4.1)
  launch_scale_fn<T>(c->fh0, c->f0, c->f0 + m, c->f0 + 2 * m, c->f0 + 3 * m, c->f0 + 4 * m, c->D, true, m, c->fh, fsp,
                     fsp + m, fsp + 2 * m, fsp + 3 * m, fsp + 4 * m, s);
  launch_scale_fn<T>(c->gh0, c->g0, c->g0 + n, c->g0 + 2 * n, c->g0 + 3 * n, c->g0 + 4 * n, c->E, false, n, c->gh, gsp,
                     gsp + n, gsp + 2 * n, gsp + 3 * n, gsp + 4 * n, s);
  return POGS_OK;
}

// An event of the calling thread on the current device, kept until the
// process ends (no event is created or destroyed per solve).  It is recorded
// and waited on within one call, so contexts on the same thread share it.
hipEvent_t thread_event() {
  static thread_local std::vector<std::pair<int, hipEvent_t>> evs;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  for (auto &e : evs)
    if (e.first == dev) return e.second;
  hipEvent_t ev = nullptr;
  if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return nullptr;
  evs.push_back({dev, ev});
  return ev;
}

// Iterations per captured launch sequence: positive and even (the control
// state alternates between two buffers by iteration parity).
int even_chunk(int requested) {
  const int c = requested > 0 ? requested : 20;
  return c + (c & 1);
}

// One chunk of iterations (chunk even: iteration parity is i % 2), then the
// stop test of its last iteration so the state after the chunk is in st[0].
// cg_cap > 0 selects the CGLS projection with that step cap; gap adds the
// gap test after each prox step.
// Iterations i0 .. i1 - 1 of a chunk, and with preview the chunk's closing
// stop test (i1 = chunk).
template <typename T>
void launch_iters(pogs_ctx *c, int i0, int i1, bool preview, int cg_cap, int gap, hipStream_t s) {
  const IterArgs<T> p0 = c->iter_args<T>(0), p1 = c->iter_args<T>(c->fused ? 1 : 0);
  IterArgs<T> p = p0;
  for (int i = i0; i < i1; ++i) {
    p = (i & 1) ? p1 : p0;  // half-step set by iteration parity (one-pass iteration)
    p.par = i & 1;
    if (c->sparse) launch_iteration_cg_sparse<T>(p, cg_cap, s);
    else if (cg_cap > 0) launch_iteration_cg<T>(p, c->splits, c->rps, c->ncolp, cg_cap, s);
    else if (gap) launch_iteration_gap<T>(p, c->splits, c->rps, c->ncolp, s);
    else launch_iteration<T>(p, c->splits, c->rps, c->ncolp, s);
  }
  if (preview) {
    p = p1;
    p.par = 1;
    launch_control_preview<T>(p, 1, s);
  }
}
template <typename T> void launch_chunk(pogs_ctx *c, int chunk, int cg_cap, int gap, hipStream_t s) {
  launch_iters<T>(c, 0, chunk, true, cg_cap, gap, s);
}

template <typename T> int ensure_graph(pogs_ctx *c, int chunk, int cg_cap, int gap) {
  if (c->graph && c->graph_chunk == chunk && c->graph_cg_cap == cg_cap && c->graph_gap == gap) return POGS_OK;
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  // captured on a stream of this thread that never runs work, so the
  // context's stream can be executing the first chunk meanwhile
  static thread_local hipStream_t cap = nullptr;
  if (!cap) POGS_HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipGraph_t g;
  POGS_HIP_TRY(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
  launch_chunk<T>(c, chunk, cg_cap, gap, cap);
  POGS_HIP_TRY(hipStreamEndCapture(cap, &g));
  hipError_t e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return POGS_EDEVICE;
  c->graph_chunk = chunk;
  c->graph_cg_cap = cg_cap;
  c->graph_gap = gap;
  return POGS_OK;
}

template <typename T> int solve_impl(pogs_ctx *c, const pogs_fn *f, const pogs_fn *g, const pogs_params &p,
                                     const void *x0, const void *nu0, pogs_result *out) {
  const double t0 = now_ms();
  const int m = (int)c->m, n = (int)c->n;
  hipStream_t s = c->stream;
  const int cg_cap = p.projection == POGS_PROJ_CGLS ? p.cg_max_iter : 0;
  const int gap = p.stop_rule == POGS_STOP_GAP ? 1 : 0;
  int rc;
  if ((rc = upload_fns<T>(c, f, g))) return rc;  // validates f and g first
  // tall float32 direct solves with the residual rule read A once per iteration
  c->fused = c->fp_blocks > 0 && cg_cap == 0 && !gap;
  // zero state (Algorithm 1 starts from x = y = x~ = y~ = 0), or the warm start
  POGS_HIP_TRY(hipMemsetAsync(c->vec, 0, c->vec_elems() * sizeof(T), s));
  if (x0 || nu0) {
    const T *dx0 = (const T *)x0, *dnu0 = (const T *)nu0;
    if (out->mem == POGS_HOST) {  // staged in the output vectors (written again at the end)
      if (x0) {
        POGS_HIP_TRY(hipMemcpyAsync(c->vecp<T>(11), x0, (size_t)n * sizeof(T), hipMemcpyHostToDevice, s));
        dx0 = c->vecp<T>(11);
      }
      if (nu0) {
        POGS_HIP_TRY(hipMemcpyAsync(c->vecp<T>(14), nu0, (size_t)m * sizeof(T), hipMemcpyHostToDevice, s));
        dnu0 = c->vecp<T>(14);
      }
    }
    if (c->sparse) launch_warm_start_sparse<T>(c->iter_args<T>(), c->D, c->E, p.rho0, dx0, dnu0, s);
    else launch_warm_start<T>(c->iter_args<T>(), c->splits, c->rps, c->ncolp, c->D, c->E, p.rho0, dx0, dnu0, s);
    if (cg_cap > 0) launch_cg_from_state<T>(c->iter_args<T>(), s);
    if (out->mem == POGS_HOST) POGS_HIP_TRY(hipStreamSynchronize(s));  // host x0, nu0 may be pageable
  }
  Ctrl h{};
  h.eps_abs = p.eps_abs;
  h.eps_rel = p.eps_rel;
  h.alpha = p.alpha;
  h.delta = p.delta;
  h.tau = p.tau;
  h.max_iter = p.max_iter;
  h.adaptive = p.adaptive_rho ? 1 : 0;
  for (int b = 0; b < 2; ++b) {  // iteration 0 reads st[1]: no stop test pending
    h.st[b].rho = p.rho0;
    h.st[b].rescale = 1.0;
  }
  h.cg_tol = p.cg_tol;
  h.cg_cap = cg_cap;
  h.stop_gap = gap;
  h.cg.stop = -1;
  *c->ctrl_host = h;
  POGS_HIP_TRY(hipMemcpyAsync(c->ctrl, c->ctrl_host, sizeof(Ctrl), hipMemcpyHostToDevice, s));
  const int chunk = even_chunk(p.chunk_iters);
  // Large problems launch every chunk directly: an iteration keeps the GPU
  // busy longer than the host takes to issue it, and a graph would only add
  // its capture and, at pogs_free, its destruction (about 1 ms for a chunk of
  // 20 iterations).  Smaller ones replay a graph; without one for this chunk
  // size yet, the first chunk is launched directly and the graph is captured
  // while the GPU runs it.
  const bool direct = c->sparse ? c->nnz >= ((int64_t)1 << 22) : (double)c->m * (double)c->n >= 16.0 * (1 << 20);
  bool eager = direct || !(c->graph && c->graph_chunk == chunk && c->graph_cg_cap == cg_cap && c->graph_gap == gap);
  // Directly launched chunks: while the host waits for a chunk's control
  // read-back, the first kLookahead iterations of the next chunk are already
  // queued, so the GPU does not idle while the host wakes and launches the
  // rest.  After the chunk that stops, they return at once (every iteration
  // kernel checks the stop flag first).
  constexpr int kLookahead = 1;
  hipEvent_t chunk_done = nullptr;
  if (direct && !(chunk_done = thread_event())) return POGS_EDEVICE;
  if (direct) launch_chunk<T>(c, chunk, cg_cap, gap, s);
  for (;;) {
    if (direct) {
      POGS_HIP_TRY(hipMemcpyAsync(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
      POGS_HIP_TRY(hipEventRecord(chunk_done, s));
      launch_iters<T>(c, 0, kLookahead, false, cg_cap, gap, s);
      POGS_HIP_TRY(hipEventSynchronize(chunk_done));
    } else {
      if (eager) launch_chunk<T>(c, chunk, cg_cap, gap, s);
      else POGS_HIP_TRY(hipGraphLaunch(c->graph, s));
      POGS_HIP_TRY(hipMemcpyAsync(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s));
      if (eager) {
        if ((rc = ensure_graph<T>(c, chunk, cg_cap, gap))) return rc;
        eager = false;
      }
      POGS_HIP_TRY(hipStreamSynchronize(s));
    }
    const CtrlState &cs = c->ctrl_host->st[0];
    if (p.verbose)
      fprintf(stderr, "pogs: k=%d r_pri=%.3e eps_pri=%.3e r_dual=%.3e eps_dual=%.3e rho=%.4g\n", cs.k, cs.r_pri,
              cs.eps_pri, cs.r_dual, cs.eps_dual, cs.rho);
    if (cs.done) break;
    if (direct) launch_iters<T>(c, kLookahead, chunk, true, cg_cap, gap, s);
  }
  // unscale into the caller's buffers (device) or staging (host); the
  // one-pass iteration left the last iteration's half step in set (k - 1) % 2
  const int last_set = c->fused ? ((c->ctrl_host->st[0].k - 1) & 1) : 0;
  const IterArgs<T> ia = c->iter_args<T>(last_set);
  T *xo = c->vecp<T>(11), *yo = c->vecp<T>(12), *muo = c->vecp<T>(13), *nuo = c->vecp<T>(14);
  if (out->mem == POGS_DEVICE) {
    xo = (T *)out->x;
    yo = (T *)out->y;
    muo = (T *)out->mu;
    nuo = (T *)out->nu;
  }
  double *fa = c->f0, *ga = c->g0;
  const CtrlState &fin = c->ctrl_host->st[0];
  launch_unscale<T>(ia, c->D, c->E, c->fh0, fa, fa + m, fa + 2 * m, fa + 3 * m, fa + 4 * m, c->gh0, ga, ga + n,
                    ga + 2 * n, ga + 3 * n, ga + 4 * n, xo, yo, muo, nuo, ia.s_gconj + ia.nbx + ia.nby,
                    c->obj_dev, c->counters + (int)cdiv(n, gemv_t_tile(sizeof(T))) + 8, fin.by_gap,
                    fin.rho, s);
  POGS_HIP_TRY(hipMemcpyAsync(c->obj_host, c->obj_dev, sizeof(double), hipMemcpyDeviceToHost, s));
  if (out->mem == POGS_HOST) {
    if (out->x) POGS_HIP_TRY(hipMemcpyAsync(out->x, xo, (size_t)n * sizeof(T), hipMemcpyDeviceToHost, s));
    if (out->y) POGS_HIP_TRY(hipMemcpyAsync(out->y, yo, (size_t)m * sizeof(T), hipMemcpyDeviceToHost, s));
    if (out->mu) POGS_HIP_TRY(hipMemcpyAsync(out->mu, muo, (size_t)n * sizeof(T), hipMemcpyDeviceToHost, s));
    if (out->nu) POGS_HIP_TRY(hipMemcpyAsync(out->nu, nuo, (size_t)m * sizeof(T), hipMemcpyDeviceToHost, s));
  }
  POGS_HIP_TRY(hipStreamSynchronize(s));
  POGS_HIP_TRY(hipGetLastError());
  const CtrlState &r = c->ctrl_host->st[0];
  out->optval = *c->obj_host;
  out->r_pri = r.r_pri;
  out->r_dual = r.r_dual;
  out->eps_pri = r.eps_pri;
  out->eps_dual = r.eps_dual;
  out->rho = r.rho;
  out->iters = r.k;
  out->status = r.done - 1;
  out->cg_steps = c->ctrl_host->cg.steps_total;
  out->gap = gap ? r.eta : NAN;
  out->eps_gap = gap ? r.eps_gap : NAN;
  out->ms_setup = c->ms_setup;
  out->ms_solve = now_ms() - t0;
  c->solved = true;
  return POGS_OK;
}

template <typename T> int profile_impl(pogs_ctx *c, int reps, double *ms) {
  hipStream_t s = c->stream;
  Ctrl h{};
  h.eps_abs = 0.0;  // stop test never passes
  h.eps_rel = 0.0;
  h.alpha = c->params.alpha;
  h.delta = c->params.delta;
  h.tau = c->params.tau;
  h.max_iter = 0x7fffffff;
  h.adaptive = 0;
  for (int b = 0; b < 2; ++b) {
    h.st[b].rho = 1.0;
    h.st[b].rescale = 1.0;
  }
  const int cg_cap = c->proj == POGS_PROJ_CGLS ? c->params.cg_max_iter : 0;
  c->fused = c->fp_blocks > 0 && cg_cap == 0;  // the launches of a residual-rule solve
  h.cg_tol = c->params.cg_tol;
  h.cg_cap = cg_cap;
  h.cg.stop = -1;
  *c->ctrl_host = h;
  POGS_HIP_TRY(hipMemcpyAsync(c->ctrl, c->ctrl_host, sizeof(Ctrl), hipMemcpyHostToDevice, s));
  const int chunk = even_chunk(c->params.chunk_iters);
  int rc;
  if ((rc = ensure_graph<T>(c, chunk, cg_cap, 0))) return rc;
  hipEvent_t e0, e1;
  POGS_HIP_TRY(hipEventCreate(&e0));
  POGS_HIP_TRY(hipEventCreate(&e1));
  float t = 0.f;
  const int launches = (int)cdiv(reps, chunk);
  POGS_HIP_TRY(hipGraphLaunch(c->graph, s));  // warm
  POGS_HIP_TRY(hipEventRecord(e0, s));
  for (int i = 0; i < launches; ++i) POGS_HIP_TRY(hipGraphLaunch(c->graph, s));
  POGS_HIP_TRY(hipEventRecord(e1, s));
  POGS_HIP_TRY(hipEventSynchronize(e1));
  POGS_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
  ms[0] = (double)t / ((double)launches * chunk);
  const IterArgs<T> p = c->iter_args<T>();
  auto part = [&](int w) {
    if (c->sparse) launch_iteration_cg_sparse_part<T>(p, w, s);
    else if (cg_cap > 0) launch_iteration_cg_part<T>(p, w, c->splits, c->rps, c->ncolp, s);
    else launch_iteration_part<T>(p, w, c->splits, c->rps, c->ncolp, s);
  };
  ms[4] = 0.0;
  for (int w = 0; w < (cg_cap > 0 ? 3 : 4); ++w) {
    if (w == 0 && p.fused) {  // no prox launch: the prox step is inside pass 1
      ms[1] = 0.0;
      continue;
    }
    part(w);  // warm
    POGS_HIP_TRY(hipEventRecord(e0, s));
    for (int i = 0; i < reps; ++i) part(w);
    POGS_HIP_TRY(hipEventRecord(e1, s));
    POGS_HIP_TRY(hipEventSynchronize(e1));
    POGS_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    ms[1 + w] = (double)t / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  POGS_HIP_TRY(hipGetLastError());
  return POGS_OK;
}

}  // namespace

extern "C" int pogs_solve(pogs_ctx *ctx, const pogs_fn *f, const pogs_fn *g, const pogs_params *params,
                          const void *x0, const void *nu0, pogs_result *out) {
  if (!ctx || !f || !g || !out) return POGS_EINVAL;

  if (out->mem != POGS_HOST && out->mem != POGS_DEVICE) return POGS_EINVAL;
  pogs_params p = params ? *params : ctx->params;
  if (check_params(p)) return POGS_EINVAL;
  if (ctx->sparse) p.projection = POGS_PROJ_CGLS;  // a sparse context always projects by CGLS
  // a context set up for CGLS has no factor for the direct projection; the
  // CGLS state does not keep x~ and y~ for the gap test
  if (p.projection == POGS_PROJ_DIRECT && ctx->proj != POGS_PROJ_DIRECT) return POGS_EUNSUPPORTED;
  if (p.projection == POGS_PROJ_CGLS && p.stop_rule == POGS_STOP_GAP) return POGS_EUNSUPPORTED;
  return ctx->dt == POGS_F32 ? solve_impl<float>(ctx, f, g, p, x0, nu0, out)
                             : solve_impl<double>(ctx, f, g, p, x0, nu0, out);
}

extern "C" int pogs_profile_iteration(pogs_ctx *ctx, int32_t reps, double *ms) {
  if (!ctx || reps < 1 || !ms || !ctx->solved) return POGS_EINVAL;
  return ctx->dt == POGS_F32 ? profile_impl<float>(ctx, reps, ms) : profile_impl<double>(ctx, reps, ms);
}

extern "C" int pogs_get_scaling(pogs_ctx *ctx, double *D, double *E, pogs_mem mem) {
  if (!ctx || (mem != POGS_HOST && mem != POGS_DEVICE)) return POGS_EINVAL;
  const hipMemcpyKind k = mem == POGS_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  if (D) POGS_HIP_TRY(hipMemcpyAsync(D, ctx->D, (size_t)ctx->m * 8, k, ctx->stream));
  if (E) POGS_HIP_TRY(hipMemcpyAsync(E, ctx->E, (size_t)ctx->n * 8, k, ctx->stream));
  POGS_HIP_TRY(hipStreamSynchronize(ctx->stream));
  return POGS_OK;
}

namespace {
template <typename T> int project_impl(pogs_ctx *c, const void *cv, const void *dv, void *x, void *y, pogs_mem mem) {
  if (c->proj != POGS_PROJ_DIRECT) return POGS_EUNSUPPORTED;
  const int m = (int)c->m, n = (int)c->n;
  hipStream_t s = c->stream;
  // inputs/outputs staged in the output vectors 11..14 when on the host
  const T *cin = (const T *)cv, *din = (const T *)dv;
  T *xo = (T *)x, *yo = (T *)y;
  if (mem == POGS_HOST) {
    T *cs = c->vecp<T>(13), *ds = c->vecp<T>(14);
    POGS_HIP_TRY(hipMemcpyAsync(cs, cv, (size_t)n * sizeof(T), hipMemcpyHostToDevice, s));
    POGS_HIP_TRY(hipMemcpyAsync(ds, dv, (size_t)m * sizeof(T), hipMemcpyHostToDevice, s));
    cin = cs;
    din = ds;
    xo = c->vecp<T>(11);
    yo = c->vecp<T>(12);
  }
  launch_project<T>(c->iter_args<T>(), c->splits, c->rps, c->ncolp, cin, din, xo, yo, s);
  if (mem == POGS_HOST) {
    POGS_HIP_TRY(hipMemcpyAsync(x, xo, (size_t)n * sizeof(T), hipMemcpyDeviceToHost, s));
    POGS_HIP_TRY(hipMemcpyAsync(y, yo, (size_t)m * sizeof(T), hipMemcpyDeviceToHost, s));
  }
  POGS_HIP_TRY(hipStreamSynchronize(s));
  POGS_HIP_TRY(hipGetLastError());
  return POGS_OK;
}

template <typename T> int prox_impl(const HostFn &F, double rho, const void *v, void *out, pogs_mem mem,
                                    hipStream_t s) {
  const int L = (int)F.h.size();
  DevArena tmp(s);
  int rc;
  uint8_t *h;
  T *prm, *vd, *od;
  if ((rc = tmp.alloc((void **)&h, L))) return rc;
  if ((rc = tmp.alloc((void **)&prm, (size_t)5 * L * sizeof(T)))) return rc;
  std::vector<T> hp((size_t)5 * L);
  const std::vector<double> *arr[5] = {&F.a, &F.b, &F.c, &F.d, &F.e};
  for (int j = 0; j < 5; ++j)
    for (int i = 0; i < L; ++i) hp[(size_t)j * L + i] = (T)(*arr[j])[i];
  POGS_HIP_TRY(hipMemcpyAsync(h, F.h.data(), L, hipMemcpyHostToDevice, s));
  POGS_HIP_TRY(hipMemcpyAsync(prm, hp.data(), hp.size() * sizeof(T), hipMemcpyHostToDevice, s));
  if (mem == POGS_HOST) {
    if ((rc = tmp.alloc((void **)&vd, (size_t)L * sizeof(T)))) return rc;
    if ((rc = tmp.alloc((void **)&od, (size_t)L * sizeof(T)))) return rc;
    POGS_HIP_TRY(hipMemcpyAsync(vd, v, (size_t)L * sizeof(T), hipMemcpyHostToDevice, s));
  } else {
    vd = (T *)v;
    od = (T *)out;
  }
  launch_prox_eval<T>(h, prm, prm + L, prm + 2 * L, prm + 3 * L, prm + 4 * L, rho, vd, od, L, s);
  if (mem == POGS_HOST) POGS_HIP_TRY(hipMemcpyAsync(out, od, (size_t)L * sizeof(T), hipMemcpyDeviceToHost, s));
  POGS_HIP_TRY(hipStreamSynchronize(s));
  POGS_HIP_TRY(hipGetLastError());
  return POGS_OK;
}
}  // namespace

extern "C" int pogs_project(pogs_ctx *ctx, const void *c, const void *d, void *x, void *y, pogs_mem mem) {
  if (!ctx || !c || !d || !x || !y || (mem != POGS_HOST && mem != POGS_DEVICE)) return POGS_EINVAL;
  return ctx->dt == POGS_F32 ? project_impl<float>(ctx, c, d, x, y, mem) : project_impl<double>(ctx, c, d, x, y, mem);
}

extern "C" int pogs_prox(const pogs_fn *fn, pogs_dtype dt, double rho, const void *v, void *out, pogs_mem mem,
                         void *stream) {
  if (!fn || !v || !out || fn->len <= 0 || !(rho > 0.0) || !std::isfinite(rho)) return POGS_EINVAL;
  if ((dt != POGS_F32 && dt != POGS_F64) || (mem != POGS_HOST && mem != POGS_DEVICE)) return POGS_EINVAL;
  HostFn F;
  int rc;
  if ((rc = expand_fn(fn, fn->len, &F))) return rc;
  hipStream_t s = (hipStream_t)stream;
  return dt == POGS_F32 ? prox_impl<float>(F, rho, v, out, mem, s) : prox_impl<double>(F, rho, v, out, mem, s);
}
