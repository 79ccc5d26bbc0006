// Host side of the batched solver and the serving engine, on top of the
// grouped launches (group_engine.hpp): every launch runs one phase for all
// problems of a group, so each pass over a matrix has the whole GPU behind it.
//
// Serving (continuous batching): a scheduler thread admits queued requests
// while the resident set fits the memory budget and the slot count, runs the
// setup of the newly admitted ones as one group, then one chunk of
// chunk_iters iterations of every resident problem.  Finished problems are
// returned and their memory released after each chunk, so requests that
// arrive while others are on the GPU join at the next chunk.  Problems too
// large for the grouped path, or large enough to slow every chunk, run on the
// whole-GPU path on two more threads (one stream each), overlapping the chunks.
#include <algorithm>
#include <atomic>
#include <cfloat>
#include <cmath>
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

#include "ctx.hpp"
#include "group_engine.hpp"
#include "hostutil.hpp"
#include "upload.hpp"

using namespace pogs;

namespace {

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// A validated, self-contained copy of one problem (host memory).
struct HostProblem {
  int m = 0, n = 0;
  std::unique_ptr<float[]> A;  // row-major m x n
  HostFn f, g;
  pogs_params params{};
};

// Validate a problem (not its matrix entries).
int check_problem(const pogs_problem *p) {
  if (!p || p->m <= 0 || p->n <= 0 || !p->A) return POGS_EINVAL;
  if (p->m > (1LL << 31) - 1 || p->n > (1LL << 31) - 1) return POGS_EINVAL;
  if (p->dt != POGS_F32) return POGS_EUNSUPPORTED;
  if (p->ord != POGS_ROW_MAJOR && p->ord != POGS_COL_MAJOR) return POGS_EINVAL;
  if (p->lda < (p->ord == POGS_ROW_MAJOR ? p->n : p->m)) return POGS_EINVAL;
  if (check_params(p->params)) return POGS_EINVAL;
  // grouped path: cached factors and the residual test
  if (p->params.projection != POGS_PROJ_DIRECT || p->params.stop_rule != POGS_STOP_RESIDUAL) return POGS_EUNSUPPORTED;
  return POGS_OK;
}

// A self-contained copy (serving: the caller may free its buffers on return);
// the matrix is copied row-major and checked for non-finite entries in the
// same pass.
int make_host_problem(const pogs_problem *p, HostProblem *hp) {
  int rc;
  if ((rc = check_problem(p))) return rc;
  if ((rc = expand_fn(&p->f, p->m, &hp->f))) return rc;
  if ((rc = expand_fn(&p->g, p->n, &hp->g))) return rc;
  hp->m = (int)p->m;
  hp->n = (int)p->n;
  hp->params = p->params;
  const int64_t m = p->m, n = p->n, lda = p->lda;
  hp->A.reset(new (std::nothrow) float[(size_t)m * n]);  // not zero-filled: every entry is written below
  if (!hp->A) return POGS_ENOMEM;
  const float *src = (const float *)p->A;
  float *dst = hp->A.get();
  const bool rowmajor = p->ord == POGS_ROW_MAJOR;
  // copy and check in one pass over row ranges, on the host pool's threads
  // for large matrices; a non-finite float has all exponent bits set
  const int parts = (size_t)m * n >= ((size_t)1 << 20) ? 16 : 1;
  std::atomic<unsigned> bad{0};
  auto body = [&](int part) {
    const int64_t i0 = m * part / parts, i1 = m * (part + 1) / parts;
    unsigned nb = 0;
    for (int64_t i = i0; i < i1; ++i) {
      float *d = dst + i * n;
      if (rowmajor) {
        const float *r = src + i * lda;
        for (int64_t j = 0; j < n; ++j) {
          const float v = r[j];
          d[j] = v;
          uint32_t b;
          std::memcpy(&b, &v, 4);
          nb |= (b & 0x7f800000u) == 0x7f800000u;
        }
      } else {
        for (int64_t j = 0; j < n; ++j) {
          const float v = src[j * lda + i];
          d[j] = v;
          uint32_t b;
          std::memcpy(&b, &v, 4);
          nb |= (b & 0x7f800000u) == 0x7f800000u;
        }
      }
    }
    if (nb) bad = 1;
  };
  if (parts > 1) host_pool().run(parts, body);
  else body(0);
  return bad ? POGS_EINVAL : POGS_OK;
}

// Problems the batch call and the serving engine run on the whole-GPU path:
// those the grouped path does not take, and those large enough to slow every
// chunk of the group (their passes and Gram tiles would run on a few CUs).
bool serve_solo(int m, int n) {
  return !GroupEngine::fits(m, n) || (double)m * n > 16.0 * (1 << 20) || std::min(m, n) > 2048;
}

void fill_result(const GStatus &st, pogs_result *out, double ms_solve) {
  const CtrlState &c = st.st;
  out->optval = st.obj;
  out->r_pri = c.r_pri;
  out->r_dual = c.r_dual;
  out->eps_pri = c.eps_pri;
  out->eps_dual = c.eps_dual;
  out->rho = c.rho;
  out->iters = c.k;
  out->status = st.flags[1] ? POGS_NUMERICAL : (c.done ? c.done - 1 : POGS_MAXITER);
  out->ms_setup = 0.0;
  out->ms_solve = ms_solve;
  out->cg_steps = 0;
  out->gap = NAN;
  out->eps_gap = NAN;
}

// Whole-GPU path for one problem (used for problems too large for a workgroup).
int solve_large(const HostProblem &hp, pogs_result *out, hipStream_t s) {
  pogs_ctx *ctx = nullptr;
  int rc = pogs_init(&ctx, hp.m, hp.n, hp.A.get(), POGS_F32, POGS_ROW_MAJOR, hp.n, POGS_HOST, &hp.params, s);
  if (rc) return rc;
  std::vector<uint8_t> fh(hp.f.h), gh(hp.g.h);
  pogs_fn f{hp.m, 1, fh.data(), hp.f.a.data(), hp.f.b.data(), hp.f.c.data(), hp.f.d.data(), hp.f.e.data()};
  pogs_fn g{hp.n, 1, gh.data(), hp.g.a.data(), hp.g.b.data(), hp.g.c.data(), hp.g.d.data(), hp.g.e.data()};
  rc = pogs_solve(ctx, &f, &g, &hp.params, nullptr, nullptr, out);
  pogs_free(ctx);
  return rc;
}

}  // namespace

// ---------------------------------------------------------------------------
// One-call batch
// ---------------------------------------------------------------------------
extern "C" int pogs_solve_batch(int32_t nprob, const pogs_problem *probs, pogs_result *out, void *stream) {
  if (nprob <= 0 || !probs || !out) return POGS_EINVAL;
  const double t0 = now_ms();
  std::vector<HostFn> fs(nprob), gs(nprob);
  for (int i = 0; i < nprob; ++i) {
    int rc = check_problem(&probs[i]);
    if (!rc) rc = expand_fn(&probs[i].f, probs[i].m, &fs[i]);
    if (!rc) rc = expand_fn(&probs[i].g, probs[i].n, &gs[i]);
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
  std::vector<int> grouped, large;
  for (int i = 0; i < nprob; ++i)
    (serve_solo((int)probs[i].m, (int)probs[i].n) ? large : grouped).push_back(i);
  int rc;
  if (!grouped.empty()) {
    GroupEngine eng(s, (int)grouped.size());
    if ((rc = eng.init())) return rc;
    std::vector<int> handle(nprob, -1), active;
    int chunk = 0;
    const bool verbose = probs[grouped[0]].params.verbose != 0;
    double t_add = 0.0, t_setup = 0.0, t_chunks = 0.0, t_out = 0.0;
    int nchunks = 0;
    double tp = now_ms();
    // one block for every problem's persistent arrays and one for the setup
    // workspaces (released once the setup has run)
    std::vector<size_t> off_a(grouped.size()), off_w(grouped.size());
    size_t tot_a = 0, tot_w = 0;
    for (size_t k = 0; k < grouped.size(); ++k) {
      size_t a, w;
      GroupEngine::split_bytes((int)probs[grouped[k]].m, (int)probs[grouped[k]].n, &a, &w);
      off_a[k] = tot_a;
      off_w[k] = tot_w;
      tot_a += round_up(a, 256);
      tot_w += round_up(w, 256);
    }
    DevArena blocks(s);
    char *blk_a, *blk_w;
    if ((rc = blocks.alloc((void **)&blk_a, tot_a))) return rc;
    if ((rc = blocks.alloc((void **)&blk_w, tot_w))) return rc;
    POGS_HIP_TRY(hipMemsetAsync(blk_a, 0, tot_a, s));
    POGS_HIP_TRY(host_uploader().order(s));  // the matrix uploads below go into blk_w
    size_t k = 0;
    for (int i : grouped) {
      const pogs_problem &p = probs[i];
      GroupEngine::Input in;
      in.arena = blk_a + off_a[k];
      in.ws = blk_w + off_w[k];
      ++k;
      in.m = (int)p.m;
      in.n = (int)p.n;
      in.A = (const float *)p.A;
      in.colmajor = p.ord == POGS_COL_MAJOR;
      in.lda = p.lda;
      in.f = &fs[i];
      in.g = &gs[i];
      in.params = p.params;
      if ((rc = eng.add(in, &handle[i]))) return rc;
      active.push_back(handle[i]);
      chunk = std::max(chunk, p.params.chunk_iters > 0 ? p.params.chunk_iters : 20);
    }
    t_add = now_ms() - tp;
    tp = now_ms();
    if ((rc = eng.setup(active))) return rc;
    blocks.release(blk_w);
    t_setup = now_ms() - tp;
    for (int h : active)
      if (eng.status(h).flags[0]) return POGS_EINVAL;  // non-finite entries in A
    std::vector<int> index_of(grouped.size());
    for (int i : grouped) index_of[handle[i]] = i;
    while (!active.empty()) {
      tp = now_ms();
      if ((rc = eng.run_chunk(active, chunk))) return rc;
      t_chunks += now_ms() - tp;
      ++nchunks;
      if (verbose)
        fprintf(stderr, "pogs batch: chunk %d, %zu problems, %.2f ms\n", nchunks, active.size(), now_ms() - tp);
      tp = now_ms();
      std::vector<int> done, still;
      for (int h : active) (eng.status(h).st.done || eng.status(h).flags[1] ? done : still).push_back(h);
      if (!done.empty()) {
        if ((rc = eng.finish(done))) return rc;
        std::vector<pogs_result *> outs;
        for (int h : done) outs.push_back(&out[index_of[h]]);
        if ((rc = eng.copy_out_many(done, outs))) return rc;
        for (int h : done) {
          fill_result(eng.status(h), &out[index_of[h]], now_ms() - t0);
          eng.remove(h);
        }
      }
      active.swap(still);
      t_out += now_ms() - tp;
    }
    POGS_HIP_TRY(hipStreamSynchronize(s));
    if (verbose)
      fprintf(stderr, "pogs batch: %zu grouped problems: add %.1f ms, setup %.1f ms, %d chunks %.1f ms, results %.1f ms\n",
              grouped.size(), t_add, t_setup, nchunks, t_chunks, t_out);
  }
  for (int i : large) {
    HostProblem hp;
    if ((rc = make_host_problem(&probs[i], &hp))) return rc;
    if ((rc = solve_large(hp, &out[i], s))) return rc;
  }
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
  int handle = -1;  // grouped engine handle while resident
  pogs_result res{};
  std::vector<float> xo, yo, muo, nuo;
  double t_submit = 0.0;
};

}  // namespace

struct pogs_batch {
  pogs_batch_cfg cfg{};
  // requests for the whole-GPU path run on kSolo threads, each with its own
  // stream, so a short one does not wait behind a long one
  static constexpr int kSolo = 2;
  hipStream_t stream = nullptr, solo_stream[kSolo] = {};
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
  std::unique_ptr<GroupEngine> eng;
  std::thread worker, solo[kSolo];
  int error = 0;

  void run();
  void run_solo(int w);
  // status_override >= 0 replaces the result's status; err != 0 marks a
  // request whose setup failed (status POGS_FAILED, the code in res.error)
  void finish(const std::shared_ptr<Request> &r, int status_override, int err = 0);
  // bytes the request at the head of the whole-GPU queue waits for (the
  // grouped admission leaves them free so that request is not starved)
  size_t solo_wait = 0;
};

void pogs_batch::finish(const std::shared_ptr<Request> &r, int status_override, int err) {
  std::lock_guard<std::mutex> g(mu);
  if (status_override >= 0) r->res.status = status_override;
  if (err) {
    r->res.status = POGS_FAILED;
    r->res.error = err;
  }
  r->state = 2;
  if (r->bytes) used -= r->bytes;
  --pending;
  cv_done.notify_all();
  cv.notify_all();
}

void pogs_batch::run() {
  int free_slots = cfg.max_slots;
  for (;;) {
    std::vector<std::shared_ptr<Request>> admitted;
    {
      std::unique_lock<std::mutex> lk(mu);
      // wake for resident work, or for a queued request that can be admitted
      // now (memory held by whole-GPU requests is released by finish())
      cv.wait(lk, [&] {
        if (stop || !resident.empty()) return true;
        if (queue.empty() || free_slots <= 0) return false;
        const auto &h = queue.front();
        return h->cancel || used + h->bytes + solo_wait <= budget;
      });
      if (stop) return;
      // admit while memory and slots allow (first come, first served)
      while (!queue.empty() && free_slots > 0) {
        auto r = queue.front();
        if (r->cancel) {
          queue.pop_front();
          r->res.status = POGS_CANCELLED;
          r->state = 2;
          --pending;
          cv_done.notify_all();
          continue;
        }
        if (used + r->bytes + solo_wait > budget) break;
        queue.pop_front();
        used += r->bytes;
        --free_slots;
        r->state = 1;
        admitted.push_back(r);
      }
    }
    // upload and set up the newly admitted requests as one group
    std::vector<int> fresh;
    std::vector<std::shared_ptr<Request>> fresh_req;
    for (auto &r : admitted) {
      GroupEngine::Input in;
      in.m = r->hp.m;
      in.n = r->hp.n;
      in.A = r->hp.A.get();
      in.lda = r->hp.n;
      in.f = &r->hp.f;
      in.g = &r->hp.g;
      in.params = r->hp.params;
      const int rc = eng->add(in, &r->handle);
      if (rc) {
        ++free_slots;
        r->handle = -1;
        finish(r, -1, rc);
        continue;
      }
      fresh.push_back(r->handle);
      fresh_req.push_back(r);
    }
    int rc = eng->setup(fresh);
    for (auto &r : fresh_req) {
      if (rc || eng->status(r->handle).flags[0]) {
        eng->remove(r->handle);
        ++free_slots;
        finish(r, -1, rc ? rc : POGS_EINVAL);  // flags[0]: non-finite entries found on the device
        continue;
      }
      std::lock_guard<std::mutex> g(mu);
      resident.push_back(r);
    }
    if (rc) {
      std::lock_guard<std::mutex> g(mu);
      error = rc;
    }
    std::vector<std::shared_ptr<Request>> live;
    {
      std::lock_guard<std::mutex> g(mu);
      live = resident;
    }
    if (live.empty()) continue;
    // one chunk: every resident problem advances by chunk_iters iterations
    std::vector<int> hs;
    for (auto &r : live) hs.push_back(r->handle);
    rc = eng->run_chunk(hs, cfg.chunk_iters);
    std::vector<std::shared_ptr<Request>> done;
    std::vector<int> done_h;
    for (auto &r : live) {
      const GStatus &st = eng->status(r->handle);
      if (rc || st.st.done || st.flags[1] || r->cancel) {
        done.push_back(r);
        if (!r->cancel && !rc) done_h.push_back(r->handle);
      }
    }
    if (!rc && !done_h.empty()) rc = eng->finish(done_h);
    if (rc) {
      std::lock_guard<std::mutex> g(mu);
      error = rc;
    }
    for (auto &r : done) {
      const int m = r->hp.m, n = r->hp.n;
      fill_result(eng->status(r->handle), &r->res, now_ms() - r->t_submit);
      if (!rc && !r->cancel) {
        r->xo.resize(n);
        r->yo.resize(m);
        r->muo.resize(n);
        r->nuo.resize(m);
        (void)eng->copy_out(r->handle, r->xo.data(), r->yo.data(), r->muo.data(), r->nuo.data(), POGS_HOST);
      }
      eng->remove(r->handle);
      ++free_slots;
      {
        std::lock_guard<std::mutex> g(mu);
        resident.erase(std::find(resident.begin(), resident.end(), r));
      }
      finish(r, r->cancel ? POGS_CANCELLED : -1, rc);
    }
  }
}

void pogs_batch::run_solo(int w) {
  for (;;) {
    std::shared_ptr<Request> r;
    {
      // the head of the queue starts once its estimated device memory fits
      // the budget next to everything resident (grouped and whole-GPU)
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        cv.wait(lk, [&] { return stop || !solo_queue.empty(); });
        if (stop) return;
        r = solo_queue.front();
        if (r->cancel) {
          solo_queue.pop_front();
          if (solo_wait && solo_queue.empty()) solo_wait = 0;
          r->state = 2;
          r->res.status = POGS_CANCELLED;
          --pending;
          cv_done.notify_all();
          cv.notify_all();
          continue;
        }
        if (used + r->bytes <= budget) break;
        solo_wait = r->bytes;
        cv.wait(lk);
      }
      solo_queue.pop_front();
      solo_wait = 0;
      used += r->bytes;
      r->state = 1;
      cv.notify_all();
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
    const int rc = solve_large(r->hp, &r->res, solo_stream[w]);
    r->res.ms_solve = now_ms() - r->t_submit;
    finish(r, -1, rc);
  }
}

extern "C" int pogs_batch_create(pogs_batch **out, const pogs_batch_cfg *cfg) {
  if (!out) return POGS_EINVAL;
  *out = nullptr;
  std::unique_ptr<pogs_batch> b(new (std::nothrow) pogs_batch());
  if (!b) return POGS_ENOMEM;
  if (cfg) b->cfg = *cfg;
  if (b->cfg.max_slots <= 0) b->cfg.max_slots = 1024;
  if (b->cfg.chunk_iters <= 0) b->cfg.chunk_iters = 20;
  if (b->cfg.stream) {
    b->stream = (hipStream_t)b->cfg.stream;
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) return POGS_EDEVICE;
    b->own_stream = true;
  }
  for (int w = 0; w < pogs_batch::kSolo; ++w)
    if (hipStreamCreateWithFlags(&b->solo_stream[w], hipStreamNonBlocking) != hipSuccess) return POGS_EDEVICE;
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) return POGS_EDEVICE;
  b->budget = b->cfg.hbm_budget_bytes ? b->cfg.hbm_budget_bytes : (size_t)(0.8 * (double)fr);
  // the engine's own arrays: descriptors, status, work lists
  b->fixed = (size_t)b->cfg.max_slots * (sizeof(GProb) + sizeof(GStatus) + 64 * sizeof(GItem)) + (1 << 20);
  if (b->fixed >= b->budget) return POGS_EAGAIN;
  b->budget -= b->fixed;
  b->eng.reset(new (std::nothrow) GroupEngine(b->stream, b->cfg.max_slots));
  if (!b->eng) return POGS_ENOMEM;
  int rc;
  if ((rc = b->eng->init())) return rc;
  b->worker = std::thread([p = b.get()] { p->run(); });
  for (int w = 0; w < pogs_batch::kSolo; ++w) b->solo[w] = std::thread([p = b.get(), w] { p->run_solo(w); });
  *out = b.release();
  return POGS_OK;
}

extern "C" int pogs_batch_submit(pogs_batch *b, const pogs_problem *p, uint64_t *ticket) {
  if (!b || !p || !ticket) return POGS_EINVAL;
  auto r = std::make_shared<Request>();
  int rc = make_host_problem(p, &r->hp);
  if (rc) return rc;
  r->large = serve_solo(r->hp.m, r->hp.n);
  if (!r->large) {
    r->bytes = GroupEngine::bytes_for(r->hp.m, r->hp.n);
    if (r->bytes > b->budget) return POGS_EAGAIN;
  } else {
    // the whole-GPU path's device memory: the matrix, the float64 Gram and
    // factor workspace and K^-1, plus the vectors (charged while it runs)
    const size_t q = std::min(r->hp.m, r->hp.n);
    r->bytes = (size_t)r->hp.m * round_up(r->hp.n, 64) * 4 + 3 * q * q * 8 +
               (size_t)64 * (r->hp.m + r->hp.n) * 8;
    if (r->bytes > b->budget) return POGS_EAGAIN;
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
  for (auto &t : b->solo)
    if (t.joinable()) t.join();
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  for (hipStream_t &ss : b->solo_stream)
    if (ss) {
      (void)hipStreamSynchronize(ss);
      (void)hipStreamDestroy(ss);
    }
  b->eng.reset();
  if (b->own_stream && b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return POGS_OK;
}
