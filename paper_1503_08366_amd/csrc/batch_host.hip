// Host side of the batched solver: packing problems into device memory, the
// one-call batch entry point, and the serving engine (continuous batching).
//
// Serving: a scheduler thread admits queued requests while the resident set
// fits the memory budget and the slot count, uploads them, and runs rounds of
// the persistent batch kernel (each round: setup of new problems, then at most
// chunk_iters iterations of every resident problem).  Finished problems are
// copied out and their memory released after each round, so requests that
// arrive while others are on the GPU join at the next round.  Problems too
// large for one workgroup (min(m, n) > kBatchMaxQ or n > kBatchMaxN) run on
// the whole-GPU path on a second thread and stream, overlapping the rounds.
#include <algorithm>
#include <cfloat>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "hostutil.hpp"

using namespace pogs;

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// A validated, self-contained copy of one problem (host memory).
struct HostProblem {
  int m = 0, n = 0;
  std::vector<float> A;  // row-major m x n
  HostFn f, g;
  pogs_params params{};
};

int make_host_problem(const pogs_problem *p, HostProblem *hp) {
  if (!p || p->m <= 0 || p->n <= 0 || !p->A) return POGS_EINVAL;
  if (p->m > (1LL << 31) - 1 || p->n > (1LL << 31) - 1) return POGS_EINVAL;
  if (p->dt != POGS_F32) return POGS_EUNSUPPORTED;
  if (p->ord != POGS_ROW_MAJOR && p->ord != POGS_COL_MAJOR) return POGS_EINVAL;
  if (p->lda < (p->ord == POGS_ROW_MAJOR ? p->n : p->m)) return POGS_EINVAL;
  if (check_params(p->params)) return POGS_EINVAL;
  int rc;
  if ((rc = expand_fn(&p->f, p->m, &hp->f))) return rc;
  if ((rc = expand_fn(&p->g, p->n, &hp->g))) return rc;
  hp->m = (int)p->m;
  hp->n = (int)p->n;
  hp->params = p->params;
  hp->A.resize((size_t)p->m * p->n);
  const float *src = (const float *)p->A;
  if (p->ord == POGS_ROW_MAJOR) {
    for (int64_t i = 0; i < p->m; ++i) memcpy(&hp->A[(size_t)i * p->n], src + i * p->lda, (size_t)p->n * 4);
  } else {
    for (int64_t i = 0; i < p->m; ++i)
      for (int64_t j = 0; j < p->n; ++j) hp->A[(size_t)i * p->n + j] = src[j * p->lda + i];
  }
  for (float v : hp->A)
    if (!std::isfinite(v)) return POGS_EINVAL;
  return POGS_OK;
}

bool fits_workgroup(int m, int n) { return std::min(m, n) <= kBatchMaxQ && n <= kBatchMaxN; }

// Device footprint of one problem on the workgroup path (bytes, 256-aligned pieces).
struct Layout {
  size_t A, Kinv, D, E, f0, g0, fh, gh, fs, gs, vec, out, total;
};

size_t al(size_t b) { return (b + 255) & ~(size_t)255; }

Layout layout_of(int m, int n) {
  Layout L{};
  const size_t ld = round_up(n, 64), q = std::min(m, n), ldk = round_up(q, 64);
  const size_t ldn = round_up(n, 64), ldm = round_up(m, 64);
  size_t o = 0;
  L.A = o; o += al((size_t)m * ld * 4);
  L.Kinv = o; o += al(q * ldk * 4);
  L.D = o; o += al((size_t)m * 8);
  L.E = o; o += al((size_t)n * 8);
  L.f0 = o; o += al((size_t)5 * m * 8);
  L.g0 = o; o += al((size_t)5 * n * 8);
  L.fh = o; o += al((size_t)m);
  L.gh = o; o += al((size_t)n);
  L.fs = o; o += al((size_t)5 * m * 4);
  L.gs = o; o += al((size_t)5 * n * 4);
  L.vec = o; o += al((5 * ldn + 5 * ldm + ldk) * 4);
  L.out = o; o += al((size_t)(2 * m + 2 * n) * 4);
  L.total = o;
  return L;
}

// Upload one problem into `base` (device, L.total bytes, zeroed) and fill its descriptor.
int stage_problem(const HostProblem &hp, char *base, BProb *bp, hipStream_t s, std::vector<double> &tmp) {
  const int m = hp.m, n = hp.n;
  const Layout L = layout_of(m, n);
  const int ld = (int)round_up(n, 64), q = std::min(m, n);
  POGS_HIP_TRY(hipMemcpy2DAsync(base + L.A, (size_t)ld * 4, hp.A.data(), (size_t)n * 4, (size_t)n * 4, m,
                                hipMemcpyHostToDevice, s));
  tmp.resize((size_t)5 * (m + n));
  const std::vector<double> *fa[5] = {&hp.f.a, &hp.f.b, &hp.f.c, &hp.f.d, &hp.f.e};
  const std::vector<double> *ga[5] = {&hp.g.a, &hp.g.b, &hp.g.c, &hp.g.d, &hp.g.e};
  for (int k = 0; k < 5; ++k) memcpy(&tmp[(size_t)k * m], fa[k]->data(), (size_t)m * 8);
  for (int k = 0; k < 5; ++k) memcpy(&tmp[(size_t)5 * m + (size_t)k * n], ga[k]->data(), (size_t)n * 8);
  POGS_HIP_TRY(hipMemcpyAsync(base + L.f0, tmp.data(), (size_t)5 * m * 8, hipMemcpyHostToDevice, s));
  POGS_HIP_TRY(hipMemcpyAsync(base + L.g0, tmp.data() + (size_t)5 * m, (size_t)5 * n * 8, hipMemcpyHostToDevice, s));
  POGS_HIP_TRY(hipMemcpyAsync(base + L.fh, hp.f.h.data(), m, hipMemcpyHostToDevice, s));
  POGS_HIP_TRY(hipMemcpyAsync(base + L.gh, hp.g.h.data(), n, hipMemcpyHostToDevice, s));
  // the host staging must outlive the copies
  POGS_HIP_TRY(hipStreamSynchronize(s));
  BProb &b = *bp;
  memset(&b, 0, sizeof(b));
  b.m = m;
  b.n = n;
  b.ld = ld;
  b.q = q;
  b.ldk = (int)round_up(q, 64);
  b.Q = (int)round_up(q, 64);
  b.A = (float *)(base + L.A);
  b.Kinv = (float *)(base + L.Kinv);
  b.D = (double *)(base + L.D);
  b.E = (double *)(base + L.E);
  b.fh = (const uint8_t *)(base + L.fh);
  b.gh = (const uint8_t *)(base + L.gh);
  b.f0 = (const double *)(base + L.f0);
  b.g0 = (const double *)(base + L.g0);
  b.fs = (float *)(base + L.fs);
  b.gs = (float *)(base + L.gs);
  b.vec = (float *)(base + L.vec);
  b.out = (float *)(base + L.out);
  b.ldn = (int)round_up(n, 64);
  b.ldm = (int)round_up(m, 64);
  const pogs_params &p = hp.params;
  b.eps_abs = p.eps_abs;
  b.eps_rel = p.eps_rel;
  b.rho0 = p.rho0;
  b.alpha = p.alpha;
  b.delta = p.delta;
  b.tau = p.tau;
  const double eps = p.eps_cmp > 0.0 ? p.eps_cmp : (double)FLT_EPSILON;
  b.gamma = (double)(m + n) * std::sqrt(eps);
  b.max_iter = p.max_iter;
  b.adaptive = p.adaptive_rho ? 1 : 0;
  b.equil_iters = p.equil_iters;
  b.status = -1;
  return POGS_OK;
}

void fill_result(const BProb &b, pogs_result *out, double ms_solve) {
  out->optval = b.optval;
  out->r_pri = b.r_pri;
  out->r_dual = b.r_dual;
  out->eps_pri = b.eps_pri;
  out->eps_dual = b.eps_dual;
  out->rho = b.rho;
  out->iters = b.k;
  out->status = b.bad ? POGS_NUMERICAL : b.status;
  out->ms_setup = 0.0;
  out->ms_solve = ms_solve;
}

int copy_outputs(const char *dev_out, int m, int n, pogs_result *out, hipStream_t s) {
  const float *o = (const float *)dev_out;
  const hipMemcpyKind k = out->mem == POGS_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (out->x) POGS_HIP_TRY(hipMemcpyAsync(out->x, o, (size_t)n * 4, k, s));
  if (out->y) POGS_HIP_TRY(hipMemcpyAsync(out->y, o + n, (size_t)m * 4, k, s));
  if (out->mu) POGS_HIP_TRY(hipMemcpyAsync(out->mu, o + n + m, (size_t)n * 4, k, s));
  if (out->nu) POGS_HIP_TRY(hipMemcpyAsync(out->nu, o + 2 * n + m, (size_t)m * 4, k, s));
  return POGS_OK;
}

// Whole-GPU path for one problem (used for problems too large for a workgroup).
int solve_large(const HostProblem &hp, pogs_result *out, hipStream_t s) {
  pogs_ctx *ctx = nullptr;
  int rc = pogs_init(&ctx, hp.m, hp.n, hp.A.data(), POGS_F32, POGS_ROW_MAJOR, hp.n, POGS_HOST, &hp.params, s);
  if (rc) return rc;
  std::vector<uint8_t> fh(hp.f.h), gh(hp.g.h);
  pogs_fn f{hp.m, 1, fh.data(), hp.f.a.data(), hp.f.b.data(), hp.f.c.data(), hp.f.d.data(), hp.f.e.data()};
  pogs_fn g{hp.n, 1, gh.data(), hp.g.a.data(), hp.g.b.data(), hp.g.c.data(), hp.g.d.data(), hp.g.e.data()};
  rc = pogs_solve(ctx, &f, &g, &hp.params, nullptr, nullptr, out);
  pogs_free(ctx);
  return rc;
}

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
  }
  int alloc(size_t b) {
    if (hipMalloc(&p, std::max<size_t>(b, 256)) != hipSuccess) {
      p = nullptr;
      return POGS_ENOMEM;
    }
    return POGS_OK;
  }
};

}  // namespace

// ---------------------------------------------------------------------------
// One-call batch
// ---------------------------------------------------------------------------
extern "C" int pogs_solve_batch(int32_t nprob, const pogs_problem *probs, pogs_result *out, void *stream) {
  if (nprob <= 0 || !probs || !out) return POGS_EINVAL;
  const double t0 = now_ms();
  std::vector<HostProblem> hp(nprob);
  for (int i = 0; i < nprob; ++i) {
    int rc = make_host_problem(&probs[i], &hp[i]);
    if (rc) return rc;
    if (out[i].mem != POGS_HOST && out[i].mem != POGS_DEVICE) return POGS_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  bool own = false;
  if (!s) {
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return POGS_EDEVICE;
    own = true;
  }
  struct StreamGuard {
    hipStream_t s;
    bool own;
    ~StreamGuard() {
      if (own) (void)hipStreamDestroy(s);
    }
  } guard{s, own};
  std::vector<int> small, large;
  for (int i = 0; i < nprob; ++i) (fits_workgroup(hp[i].m, hp[i].n) ? small : large).push_back(i);
  int rc;
  if (!small.empty()) {
    std::vector<size_t> off(small.size());
    size_t total = 0;
    int Qmax = 0, nmax = 0;
    for (size_t k = 0; k < small.size(); ++k) {
      const HostProblem &p = hp[small[k]];
      off[k] = total;
      total += layout_of(p.m, p.n).total;
      Qmax = std::max(Qmax, (int)round_up(std::min(p.m, p.n), 64));
      nmax = std::max(nmax, std::max(p.n, std::min(p.m, p.n)));
    }
    const int count = (int)small.size();
    const int slots = std::min(count, 512);
    const size_t slot_doubles = batch_slot_doubles(Qmax);
    DevBuf arena, descs, scratch;
    if ((rc = arena.alloc(total))) return rc;
    if ((rc = descs.alloc(count * sizeof(BProb) + count * sizeof(int) + 256))) return rc;
    if ((rc = scratch.alloc(slots * slot_doubles * sizeof(double)))) return rc;
    POGS_HIP_TRY(hipMemsetAsync(arena.p, 0, total, s));
    std::vector<BProb> hb(count);
    std::vector<double> tmp;
    for (int k = 0; k < count; ++k)
      if ((rc = stage_problem(hp[small[k]], (char *)arena.p + off[k], &hb[k], s, tmp))) return rc;
    // largest estimated work first (setup ~ m q^2, iterations ~ m n)
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    auto cost = [&](int k) {
      const double m = hb[k].m, n = hb[k].n, q = hb[k].q;
      return m * n * 200.0 + m * q * q / 16.0;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    BProb *dprobs = (BProb *)descs.p;
    int *dorder = (int *)((char *)descs.p + count * sizeof(BProb));
    unsigned *dnext = (unsigned *)((char *)dorder + count * sizeof(int));
    POGS_HIP_TRY(hipMemcpyAsync(dprobs, hb.data(), count * sizeof(BProb), hipMemcpyHostToDevice, s));
    POGS_HIP_TRY(hipMemcpyAsync(dorder, order.data(), count * sizeof(int), hipMemcpyHostToDevice, s));
    POGS_HIP_TRY(hipMemsetAsync(dnext, 0, sizeof(unsigned), s));
    launch_batch(dprobs, dorder, count, dnext, (double *)scratch.p, slot_doubles, slots, nmax, 0x7fffffff, s);
    POGS_HIP_TRY(hipGetLastError());
    POGS_HIP_TRY(hipMemcpyAsync(hb.data(), dprobs, count * sizeof(BProb), hipMemcpyDeviceToHost, s));
    POGS_HIP_TRY(hipStreamSynchronize(s));
    const double ms = now_ms() - t0;
    for (int k = 0; k < count; ++k) {
      const int i = small[k];
      fill_result(hb[k], &out[i], ms);
      const Layout L = layout_of(hp[i].m, hp[i].n);
      if ((rc = copy_outputs((const char *)arena.p + off[k] + L.out, hp[i].m, hp[i].n, &out[i], s))) return rc;
    }
    POGS_HIP_TRY(hipStreamSynchronize(s));
  }
  for (int i : large)
    if ((rc = solve_large(hp[i], &out[i], s))) return rc;
  return POGS_OK;
}

// ---------------------------------------------------------------------------
// Serving engine
// ---------------------------------------------------------------------------
namespace {

struct Request {
  uint64_t ticket = 0;
  HostProblem hp;
  int state = 0;  // 0 queued, 1 resident, 2 done
  bool cancel = false;
  bool large = false;
  size_t bytes = 0;
  DevBuf mem;
  int slot = -1;
  pogs_result res{};
  std::vector<float> xo, yo, muo, nuo;
  double t_submit = 0.0;
};

}  // namespace

struct pogs_batch {
  pogs_batch_cfg cfg{};
  hipStream_t stream = nullptr, solo_stream = nullptr;
  bool own_stream = false;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  bool stop = false;
  uint64_t next_ticket = 1;
  std::map<uint64_t, std::shared_ptr<Request>> reqs;
  std::deque<std::shared_ptr<Request>> queue, solo_queue;
  std::vector<std::shared_ptr<Request>> resident;
  size_t budget = 0, used = 0, fixed = 0;
  int pending = 0;
  // device resources of the rounds
  DevBuf descs, scratch;
  int slots = 0;
  size_t slot_doubles = 0;
  std::thread worker, solo;
  int error = 0;

  void run();
  void run_solo();
  void finish(const std::shared_ptr<Request> &r, int status_override);
};

void pogs_batch::finish(const std::shared_ptr<Request> &r, int status_override) {
  std::lock_guard<std::mutex> g(mu);
  if (status_override >= 0) r->res.status = status_override;
  r->state = 2;
  if (r->bytes) used -= r->bytes;
  r->mem.release();
  --pending;
  cv_done.notify_all();
  cv.notify_all();
}

void pogs_batch::run() {
  std::vector<BProb> hb;
  std::vector<double> tmp;
  std::vector<int> order;
  BProb *dprobs = (BProb *)descs.p;
  int *dorder = (int *)((char *)descs.p + cfg.max_slots * sizeof(BProb));
  unsigned *dnext = (unsigned *)((char *)dorder + cfg.max_slots * sizeof(int));
  std::vector<int> free_slots(cfg.max_slots);
  std::iota(free_slots.rbegin(), free_slots.rend(), 0);
  for (;;) {
    std::vector<std::shared_ptr<Request>> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !queue.empty() || !resident.empty(); });
      if (stop) return;
      // admit while memory and slots allow (first come, first served)
      while (!queue.empty() && !free_slots.empty()) {
        auto r = queue.front();
        if (r->cancel) {
          queue.pop_front();
          r->res.status = POGS_CANCELLED;
          r->state = 2;
          --pending;
          cv_done.notify_all();
          continue;
        }
        if (used + r->bytes > budget) break;
        queue.pop_front();
        used += r->bytes;
        r->slot = free_slots.back();
        free_slots.pop_back();
        r->state = 1;
        admitted.push_back(r);
      }
    }
    for (auto &r : admitted) {
      BProb b;
      int rc = r->mem.alloc(r->bytes);
      if (!rc) rc = hipMemsetAsync(r->mem.p, 0, r->bytes, stream) == hipSuccess ? 0 : POGS_EDEVICE;
      if (!rc) rc = stage_problem(r->hp, (char *)r->mem.p, &b, stream, tmp);
      if (!rc) rc = hipMemcpyAsync(dprobs + r->slot, &b, sizeof(BProb), hipMemcpyHostToDevice, stream) == hipSuccess
                        ? 0 : POGS_EDEVICE;
      if (!rc) rc = hipStreamSynchronize(stream) == hipSuccess ? 0 : POGS_EDEVICE;
      if (rc) {
        free_slots.push_back(r->slot);
        r->res.status = POGS_NUMERICAL;
        finish(r, POGS_NUMERICAL);
        continue;
      }
      std::lock_guard<std::mutex> g(mu);
      resident.push_back(r);
    }
    std::vector<std::shared_ptr<Request>> live;
    {
      std::lock_guard<std::mutex> g(mu);
      live = resident;
    }
    if (live.empty()) continue;
    // one round: every resident problem advances by at most chunk_iters iterations
    order.clear();
    int nmax = 1, Qmax = 64;
    for (auto &r : live) {
      order.push_back(r->slot);
      nmax = std::max(nmax, std::max(r->hp.n, std::min(r->hp.m, r->hp.n)));
      Qmax = std::max(Qmax, (int)round_up(std::min(r->hp.m, r->hp.n), 64));
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      auto ra = std::find_if(live.begin(), live.end(), [&](auto &r) { return r->slot == a; });
      auto rb = std::find_if(live.begin(), live.end(), [&](auto &r) { return r->slot == b; });
      return (double)(*ra)->hp.m * (*ra)->hp.n > (double)(*rb)->hp.m * (*rb)->hp.n;
    });
    const int count = (int)order.size();
    int rc = hipMemcpyAsync(dorder, order.data(), count * sizeof(int), hipMemcpyHostToDevice, stream) == hipSuccess
                 ? 0 : POGS_EDEVICE;
    if (!rc) rc = hipMemsetAsync(dnext, 0, sizeof(unsigned), stream) == hipSuccess ? 0 : POGS_EDEVICE;
    if (!rc) {
      launch_batch(dprobs, dorder, count, dnext, (double *)scratch.p, slot_doubles, std::min(count, slots), nmax,
                   cfg.chunk_iters, stream);
      rc = hipGetLastError() == hipSuccess ? 0 : POGS_EDEVICE;
    }
    hb.resize(cfg.max_slots);
    if (!rc) rc = hipMemcpyAsync(hb.data(), dprobs, cfg.max_slots * sizeof(BProb), hipMemcpyDeviceToHost, stream) ==
                          hipSuccess ? 0 : POGS_EDEVICE;
    if (!rc) rc = hipStreamSynchronize(stream) == hipSuccess ? 0 : POGS_EDEVICE;
    if (rc) {
      std::lock_guard<std::mutex> g(mu);
      error = rc;
    }
    for (auto &r : live) {
      const BProb &b = hb[r->slot];
      const bool done = rc || b.bad || (b.setup_done && b.status >= 0) || r->cancel;
      if (!done) continue;
      fill_result(b, &r->res, now_ms() - r->t_submit);
      const int m = r->hp.m, n = r->hp.n;
      r->xo.resize(n);
      r->yo.resize(m);
      r->muo.resize(n);
      r->nuo.resize(m);
      pogs_result tmpres{};
      tmpres.mem = POGS_HOST;
      tmpres.x = r->xo.data();
      tmpres.y = r->yo.data();
      tmpres.mu = r->muo.data();
      tmpres.nu = r->nuo.data();
      if (!rc && !r->cancel) {
        const Layout L = layout_of(m, n);
        copy_outputs((const char *)r->mem.p + L.out, m, n, &tmpres, stream);
        (void)hipStreamSynchronize(stream);
      }
      {
        std::lock_guard<std::mutex> g(mu);
        resident.erase(std::find(resident.begin(), resident.end(), r));
      }
      free_slots.push_back(r->slot);
      finish(r, rc ? POGS_NUMERICAL : (r->cancel ? POGS_CANCELLED : -1));
    }
  }
}

void pogs_batch::run_solo() {
  for (;;) {
    std::shared_ptr<Request> r;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv.wait(lk, [&] { return stop || !solo_queue.empty(); });
      if (stop) return;
      r = solo_queue.front();
      solo_queue.pop_front();
      if (r->cancel) {
        r->state = 2;
        r->res.status = POGS_CANCELLED;
        --pending;
        cv_done.notify_all();
        continue;
      }
      r->state = 1;
    }
    const int m = r->hp.m, n = r->hp.n;
    r->xo.resize(n);
    r->yo.resize(m);
    r->muo.resize(n);
    r->nuo.resize(m);
    r->res.mem = POGS_HOST;
    r->res.x = r->xo.data();
    r->res.y = r->yo.data();
    r->res.mu = r->muo.data();
    r->res.nu = r->nuo.data();
    const int rc = solve_large(r->hp, &r->res, solo_stream);
    r->res.ms_solve = now_ms() - r->t_submit;
    finish(r, rc ? POGS_NUMERICAL : -1);
  }
}

extern "C" int pogs_batch_create(pogs_batch **out, const pogs_batch_cfg *cfg) {
  if (!out) return POGS_EINVAL;
  *out = nullptr;
  std::unique_ptr<pogs_batch> b(new (std::nothrow) pogs_batch());
  if (!b) return POGS_ENOMEM;
  if (cfg) b->cfg = *cfg;
  if (b->cfg.max_slots <= 0) b->cfg.max_slots = 1024;
  if (b->cfg.chunk_iters <= 0) b->cfg.chunk_iters = 50;
  if (b->cfg.stream) {
    b->stream = (hipStream_t)b->cfg.stream;
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) return POGS_EDEVICE;
    b->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&b->solo_stream, hipStreamNonBlocking) != hipSuccess) return POGS_EDEVICE;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return POGS_EDEVICE;
  b->budget = b->cfg.hbm_budget_bytes ? b->cfg.hbm_budget_bytes : (size_t)(0.8 * (double)fr);
  b->slots = 256;
  b->slot_doubles = batch_slot_doubles(kBatchMaxQ);
  const size_t sbytes = (size_t)b->slots * b->slot_doubles * sizeof(double);
  const size_t dbytes = (size_t)b->cfg.max_slots * (sizeof(BProb) + sizeof(int)) + 256;
  if (sbytes + dbytes >= b->budget) return POGS_EAGAIN;
  int rc;
  if ((rc = b->scratch.alloc(sbytes))) return rc;
  if ((rc = b->descs.alloc(dbytes))) return rc;
  b->fixed = sbytes + dbytes;
  b->budget -= b->fixed;
  b->worker = std::thread([p = b.get()] { p->run(); });
  b->solo = std::thread([p = b.get()] { p->run_solo(); });
  *out = b.release();
  return POGS_OK;
}

extern "C" int pogs_batch_submit(pogs_batch *b, const pogs_problem *p, uint64_t *ticket) {
  if (!b || !p || !ticket) return POGS_EINVAL;
  auto r = std::make_shared<Request>();
  int rc = make_host_problem(p, &r->hp);
  if (rc) return rc;
  r->large = !fits_workgroup(r->hp.m, r->hp.n);
  if (!r->large) {
    r->bytes = layout_of(r->hp.m, r->hp.n).total;
    if (r->bytes > b->budget) return POGS_EAGAIN;
  } else {
    const size_t q = std::min(r->hp.m, r->hp.n);
    const size_t est = (size_t)r->hp.m * round_up(r->hp.n, 64) * 4 + 3 * q * q * 8;
    if (est > b->budget) return POGS_EAGAIN;
  }
  r->t_submit = now_ms();
  std::lock_guard<std::mutex> g(b->mu);
  r->ticket = b->next_ticket++;
  b->reqs[r->ticket] = r;
  ++b->pending;
  (r->large ? b->solo_queue : b->queue).push_back(r);
  b->cv.notify_all();
  *ticket = r->ticket;
  return POGS_OK;
}

extern "C" int pogs_batch_poll(pogs_batch *b, uint64_t ticket, pogs_result *out) {
  if (!b || !out) return POGS_EINVAL;
  std::shared_ptr<Request> r;
  {
    std::lock_guard<std::mutex> g(b->mu);
    auto it = b->reqs.find(ticket);
    if (it == b->reqs.end()) return POGS_ENOTFOUND;
    r = it->second;
    if (r->state != 2) return 1;
    b->reqs.erase(it);
  }
  void *x = out->x, *y = out->y, *mu = out->mu, *nu = out->nu;
  const pogs_mem mem = out->mem;
  *out = r->res;
  out->x = x;
  out->y = y;
  out->mu = mu;
  out->nu = nu;
  out->mem = mem;
  if (r->res.status == POGS_CANCELLED || r->xo.empty()) return POGS_OK;
  const int m = r->hp.m, n = r->hp.n;
  if (mem == POGS_DEVICE) {
    if (x) POGS_HIP_TRY(hipMemcpy(x, r->xo.data(), (size_t)n * 4, hipMemcpyHostToDevice));
    if (y) POGS_HIP_TRY(hipMemcpy(y, r->yo.data(), (size_t)m * 4, hipMemcpyHostToDevice));
    if (mu) POGS_HIP_TRY(hipMemcpy(mu, r->muo.data(), (size_t)n * 4, hipMemcpyHostToDevice));
    if (nu) POGS_HIP_TRY(hipMemcpy(nu, r->nuo.data(), (size_t)m * 4, hipMemcpyHostToDevice));
  } else {
    if (x) memcpy(x, r->xo.data(), (size_t)n * 4);
    if (y) memcpy(y, r->yo.data(), (size_t)m * 4);
    if (mu) memcpy(mu, r->muo.data(), (size_t)n * 4);
    if (nu) memcpy(nu, r->nuo.data(), (size_t)m * 4);
  }
  return POGS_OK;
}

extern "C" int pogs_batch_wait_all(pogs_batch *b) {
  if (!b) return POGS_EINVAL;
  std::unique_lock<std::mutex> lk(b->mu);
  b->cv_done.wait(lk, [&] { return b->pending == 0 || b->error != 0; });
  return b->error;
}

extern "C" int pogs_batch_cancel(pogs_batch *b, uint64_t ticket) {
  if (!b) return POGS_EINVAL;
  std::lock_guard<std::mutex> g(b->mu);
  auto it = b->reqs.find(ticket);
  if (it == b->reqs.end()) return POGS_ENOTFOUND;
  it->second->cancel = true;
  b->cv.notify_all();
  return POGS_OK;
}

extern "C" int pogs_batch_destroy(pogs_batch *b) {
  if (!b) return POGS_OK;
  {
    std::lock_guard<std::mutex> g(b->mu);
    b->stop = true;
    b->cv.notify_all();
  }
  if (b->worker.joinable()) b->worker.join();
  if (b->solo.joinable()) b->solo.join();
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->solo_stream) {
    (void)hipStreamSynchronize(b->solo_stream);
    (void)hipStreamDestroy(b->solo_stream);
  }
  for (auto &r : b->resident) r->mem.release();
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return POGS_OK;
}
