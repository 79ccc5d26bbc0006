// Host side of the grouped launches (see group_engine.hpp).
//
// Geometry rules depend on a problem's own (m, n) only, so its work items and
// the order of its reductions are the same in any group.
#include "group_engine.hpp"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <numeric>

#include "ctx.hpp"
#include "factor.hpp"
#include "upload.hpp"

namespace pogs {

namespace {

constexpr int kLayRows = 16;   // rows per layout work item
constexpr int kGMaxDim = 4096; // largest n and min(m, n) of the grouped path

struct Geo {
  int m, n, ld, q, Q, ldk, nbt, ldn, ldm;
  bool tall;
  int lpr16, lpr16k;
  int tiles, splits, rps, ncolp;
  int nbx, nby, n_pri, n_dual, nslots;
  int eq_U, eq_rps, eq_nsplit, eq_ncolp;
  int nt, ntp;  // Gram tiles
  // persistent arena
  size_t o_A, o_Kinv, o_D, o_E, o_raw, off_gh0, off_f0, off_g0, fn_bytes, o_fh, o_gh, o_fs, o_gs, o_vec, o_part,
      o_slots, o_ctrl, o_out, o_obj, o_cnt, o_flags, arena;
  // setup workspace
  size_t w_raw, w_d, w_e, w_eqpart, w_eqslots, w_K, w_X, w_Dinv, ws;
};

Geo geo(int m, int n) {
  Geo g{};
  g.m = m;
  g.n = n;
  g.ld = (int)round_up(n, 64);
  g.q = std::min(m, n);
  g.Q = (int)round_up(g.q, 64);
  g.ldk = g.Q;
  g.nbt = g.Q / 64;
  g.ldn = (int)round_up(n, 64);
  g.ldm = (int)round_up(m, 64);
  g.tall = m >= n;
  g.lpr16 = g.ld < 512;
  g.lpr16k = g.ldk < 512;
  g.tiles = (int)cdiv(n, 256);
  g.rps = (int)std::max<int64_t>(128, round_up(cdiv(m, 64), 4));  // 32+ rows per wave: the 8-deep load loop runs
  g.splits = (int)cdiv(m, g.rps);
  g.ncolp = g.tiles * 256;
  g.nbx = (int)cdiv(n, kBlock);
  g.nby = (int)cdiv(m, kBlock);
  g.n_pri = (int)cdiv(m, g.lpr16 ? kGRows16 : kGRows64);
  g.n_dual = (int)cdiv(n, kFinishCols);
  g.nslots = 2 * (g.nbx + g.nby) + g.n_pri + g.n_dual + g.nbx + g.nby;
  g.eq_U = (int)cdiv(n, 1024);
  g.eq_rps = (int)std::max<int64_t>(8, round_up(cdiv(m, 256), 4));
  g.eq_nsplit = (int)cdiv(m, g.eq_rps);
  g.eq_ncolp = (int)round_up(n, 256);
  g.nt = (int)cdiv(g.q, kGramTB);
  g.ntp = g.nt * (g.nt + 1) / 2;
  Carve raw;
  raw.take(m);
  g.off_gh0 = raw.take(n);
  g.off_f0 = raw.take((size_t)5 * m * 8);
  g.off_g0 = raw.take((size_t)5 * n * 8);
  g.fn_bytes = raw.off;
  Carve c;
  g.o_A = c.take((size_t)m * g.ld * 4);
  g.o_Kinv = c.take((size_t)g.q * g.ldk * 4);
  g.o_D = c.take((size_t)m * 8);
  g.o_E = c.take((size_t)n * 8);
  g.o_raw = c.take(g.fn_bytes);
  g.o_fh = c.take(m);
  g.o_gh = c.take(n);
  g.o_fs = c.take((size_t)5 * m * 4);
  g.o_gs = c.take((size_t)5 * n * 4);
  g.o_vec = c.take(((size_t)5 * g.ldn + 5 * (size_t)g.ldm + g.ldk) * 4);
  g.o_part = c.take((size_t)g.splits * 2 * g.ncolp * 8);
  g.o_slots = c.take((size_t)g.nslots * 8);
  g.o_ctrl = c.take(sizeof(Ctrl));
  g.o_out = c.take((size_t)2 * (m + n) * 4);
  g.o_obj = c.take(8);
  g.o_cnt = c.take(8);
  g.o_flags = c.take(8);
  g.arena = c.off;
  Carve w;
  g.w_raw = w.take((size_t)m * n * 4);
  g.w_d = w.take((size_t)m * 8);
  g.w_e = w.take((size_t)n * 8);
  g.w_eqpart = w.take((size_t)g.eq_nsplit * g.eq_ncolp * 8);
  g.w_eqslots = w.take((size_t)g.n_dual * 8);
  g.w_K = w.take((size_t)g.Q * g.Q * 8);
  g.w_X = w.take((size_t)g.Q * g.Q * 8);
  g.w_Dinv = w.take((size_t)g.nbt * 64 * 64 * 8);
  g.ws = w.off;
  return g;
}

template <typename P> P *at(void *base, size_t off) { return reinterpret_cast<P *>((char *)base + off); }

}  // namespace

bool GroupEngine::fits(int m, int n) { return n <= kGMaxDim && std::min(m, n) <= kGMaxDim; }

size_t GroupEngine::bytes_for(int m, int n) {
  const Geo g = geo(m, n);
  return g.arena + g.ws;
}

void GroupEngine::split_bytes(int m, int n, size_t *arena, size_t *ws) {
  const Geo g = geo(m, n);
  *arena = g.arena;
  *ws = g.ws;
}

GroupEngine::GroupEngine(hipStream_t s, int capacity) : s_(s), cap_(std::max(1, capacity)) {}

GroupEngine::~GroupEngine() {
  for (int h = 0; h < (int)used_.size(); ++h)
    if (used_[h]) remove(h);
  if (probs_dev_) (void)hipFreeAsync(probs_dev_, s_);
  if (status_dev_) (void)hipFreeAsync(status_dev_, s_);
  if (items_dev_) (void)hipFreeAsync(items_dev_, s_);
  (void)hipStreamSynchronize(s_);
  if (items_copied_) (void)hipEventDestroy(items_copied_);
  if (fn_stage_event_) (void)hipEventDestroy(fn_stage_event_);
  if (desc_copied_) (void)hipEventDestroy(desc_copied_);
  if (probs_host_) (void)hipHostFree(probs_host_);
  if (status_host_) (void)hipHostFree(status_host_);
  if (items_host_) (void)hipHostFree(items_host_);
  if (fn_stage_) (void)hipHostFree(fn_stage_);
  if (out_stage_) (void)hipHostFree(out_stage_);
}

int GroupEngine::init() {
  DevArena::configure_pool();
  probs_.assign(cap_, GProb{});
  mem_.assign(cap_, Mem{});
  used_.assign(cap_, 0);
  dirty_.assign(cap_, 0);
  if (hipHostMalloc((void **)&probs_host_, (size_t)cap_ * sizeof(GProb)) != hipSuccess) return POGS_ENOMEM;
  if (hipMallocAsync((void **)&probs_dev_, (size_t)cap_ * sizeof(GProb), s_) != hipSuccess) return POGS_ENOMEM;
  if (hipMallocAsync((void **)&status_dev_, (size_t)cap_ * sizeof(GStatus), s_) != hipSuccess) return POGS_ENOMEM;
  if (hipHostMalloc((void **)&status_host_, (size_t)cap_ * sizeof(GStatus)) != hipSuccess) return POGS_ENOMEM;
  POGS_HIP_TRY(hipMemsetAsync(status_dev_, 0, (size_t)cap_ * sizeof(GStatus), s_));
  memset(status_host_, 0, (size_t)cap_ * sizeof(GStatus));
  return POGS_OK;
}

int GroupEngine::add(const Input &in, int *handle) {
  int h = -1;
  for (int i = 0; i < cap_; ++i)
    if (!used_[i]) {
      h = i;
      break;
    }
  if (h < 0) return POGS_EAGAIN;
  const int m = in.m, n = in.n;
  const Geo g = geo(m, n);
  Mem &M = mem_[h];
  if (in.arena) {  // caller-provided, already zeroed
    M.arena = in.arena;
    M.ws = in.ws;
    M.owned = false;
  } else {
    if (hipMallocAsync(&M.arena, g.arena, s_) != hipSuccess) return POGS_ENOMEM;
    if (hipMallocAsync(&M.ws, g.ws, s_) != hipSuccess) {
      (void)hipFreeAsync(M.arena, s_);
      M.arena = nullptr;
      return POGS_ENOMEM;
    }
    M.owned = true;
    POGS_HIP_TRY(hipMemsetAsync(M.arena, 0, g.arena, s_));
  }
  used_[h] = 1;
  // input matrix, compacted (row-major: lda = n; column-major: lda = m),
  // through the pinned-ring uploader (rows packed on the host side)
  float *raw = at<float>(M.ws, g.w_raw);
  const int64_t inner = in.colmajor ? m : n, outer = in.colmajor ? n : m;
  // caller-provided memory was ordered for the uploader by the caller
  POGS_HIP_TRY(host_uploader().upload_rows(raw, in.A, (size_t)inner * 4, (size_t)in.lda * 4, (size_t)outer, s_,
                                           false, M.owned));
  upload_pending_ = true;  // fenced before the next launch on s_ or the next free
  // functions: codes and a..e, packed into a pinned ring and copied in one
  // transfer; the ring is reused from the start once the last copy out of it
  // has completed
  const size_t need = round_up(g.fn_bytes, 256);
  if (fn_stage_pos_ + need > fn_stage_cap_) {
    if (fn_stage_event_) POGS_HIP_TRY(hipEventSynchronize(fn_stage_event_));
    fn_stage_pos_ = 0;
    if (need > fn_stage_cap_) {
      if (fn_stage_) (void)hipHostFree(fn_stage_);
      fn_stage_ = nullptr;
      fn_stage_cap_ = std::max<size_t>(need, 16 << 20);
      if (hipHostMalloc((void **)&fn_stage_, fn_stage_cap_) != hipSuccess) {
        fn_stage_cap_ = 0;
        return POGS_ENOMEM;
      }
    }
  }
  char *st = fn_stage_ + fn_stage_pos_;
  fn_stage_pos_ += need;
  memcpy(st, in.f->h.data(), (size_t)m);
  memcpy(st + g.off_gh0, in.g->h.data(), (size_t)n);
  const HostFn *fs[2] = {in.f, in.g};
  const size_t offs[2] = {g.off_f0, g.off_g0};
  const int lens[2] = {m, n};
  for (int k = 0; k < 2; ++k) {
    const std::vector<double> *arr[5] = {&fs[k]->a, &fs[k]->b, &fs[k]->c, &fs[k]->d, &fs[k]->e};
    for (int j = 0; j < 5; ++j)
      memcpy(st + offs[k] + (size_t)j * lens[k] * 8, arr[j]->data(), (size_t)lens[k] * 8);
  }
  POGS_HIP_TRY(hipMemcpyAsync(at<char>(M.arena, g.o_raw), st, g.fn_bytes, hipMemcpyHostToDevice, s_));
  if (!fn_stage_event_) POGS_HIP_TRY(hipEventCreateWithFlags(&fn_stage_event_, hipEventDisableTiming));
  POGS_HIP_TRY(hipEventRecord(fn_stage_event_, s_));
  // descriptor
  GProb &P = probs_[h];
  P = GProb{};
  IterArgs<float> &it = P.it;
  it.m = m;
  it.n = n;
  it.ld = g.ld;
  it.q = g.q;
  it.ldk = g.ldk;
  it.A = at<float>(M.arena, g.o_A);
  it.Kinv = at<float>(M.arena, g.o_Kinv);
  const float *fsp = at<float>(M.arena, g.o_fs), *gsp = at<float>(M.arena, g.o_gs);
  it.f = FnDev<float>{at<uint8_t>(M.arena, g.o_fh), fsp, fsp + m, fsp + 2 * m, fsp + 3 * m, fsp + 4 * m};
  it.g = FnDev<float>{at<uint8_t>(M.arena, g.o_gh), gsp, gsp + n, gsp + 2 * n, gsp + 3 * n, gsp + 4 * n};
  float *v = at<float>(M.arena, g.o_vec);
  it.x = v;
  it.xt = v + g.ldn;
  it.xh = v + 2 * (size_t)g.ldn;
  it.mu = v + 3 * (size_t)g.ldn;
  it.cx = v + 4 * (size_t)g.ldn;
  float *vm = v + 5 * (size_t)g.ldn;
  it.y = vm;
  it.yt = vm + g.ldm;
  it.yh = vm + 2 * (size_t)g.ldm;
  it.nu = vm + 3 * (size_t)g.ldm;
  it.dy = vm + 4 * (size_t)g.ldm;
  it.rhs = vm + 5 * (size_t)g.ldm;
  it.part = at<double>(M.arena, g.o_part);
  double *sl = at<double>(M.arena, g.o_slots);
  it.nbx = g.nbx;
  it.nby = g.nby;
  it.n_smu = g.nbx;
  it.n_syh = g.nby;
  it.fused = 0;
  it.s_mu = sl;
  it.s_yh = sl + 2 * g.nbx;
  it.s_pri = sl + 2 * (g.nbx + g.nby);
  it.s_dual = it.s_pri + g.n_pri;
  it.n_pri = g.n_pri;
  it.n_dual = g.n_dual;
  it.ctrl = at<Ctrl>(M.arena, g.o_ctrl);
  it.par = 0;
  P.tall = g.tall;
  P.lpr16 = g.lpr16;
  P.lpr16k = g.lpr16k;
  P.splits = g.splits;
  P.rps = g.rps;
  P.ncolp = g.ncolp;
  P.Q = g.Q;
  P.nbt = g.nbt;
  P.eq_U = g.eq_U;
  P.eq_rps = g.eq_rps;
  P.eq_nsplit = g.eq_nsplit;
  P.eq_ncolp = g.eq_ncolp;
  P.equil_iters = in.params.equil_iters;
  P.lay_rows = kLayRows;
  P.colmajor = in.colmajor ? 1 : 0;
  P.lda = in.colmajor ? m : n;
  P.raw = raw;
  P.D = at<double>(M.arena, g.o_D);
  P.E = at<double>(M.arena, g.o_E);
  P.d = at<double>(M.ws, g.w_d);
  P.e = at<double>(M.ws, g.w_e);
  P.eq_part = at<double>(M.ws, g.w_eqpart);
  P.eq_slots = at<double>(M.ws, g.w_eqslots);
  const double eps = in.params.eps_cmp > 0.0 ? in.params.eps_cmp : (double)FLT_EPSILON;
  const double gamma = (double)(m + n) * std::sqrt(eps);
  P.gamma_m = gamma / m;
  P.gamma_n = gamma / n;
  P.mf = m;
  P.nf = n;
  P.K = at<double>(M.ws, g.w_K);
  P.X = at<double>(M.ws, g.w_X);
  P.Dinv = at<double>(M.ws, g.w_Dinv);
  P.flags = at<unsigned>(M.arena, g.o_flags);
  P.fh0 = at<uint8_t>(M.arena, g.o_raw);
  P.gh0 = at<uint8_t>(M.arena, g.o_raw + g.off_gh0);
  P.f0 = at<double>(M.arena, g.o_raw + g.off_f0);
  P.g0 = at<double>(M.arena, g.o_raw + g.off_g0);
  P.out = at<float>(M.arena, g.o_out);
  P.obj = at<double>(M.arena, g.o_obj);
  P.obj_slots = sl + 2 * (g.nbx + g.nby) + g.n_pri + g.n_dual;
  P.obj_cnt = at<unsigned>(M.arena, g.o_cnt);
  P.status = status_dev_ + h;
  const pogs_params &pp = in.params;
  P.eps_abs = pp.eps_abs;
  P.eps_rel = pp.eps_rel;
  P.alpha = pp.alpha;
  P.delta = pp.delta;
  P.tau = pp.tau;
  P.rho0 = pp.rho0;
  P.max_iter = pp.max_iter;
  P.adaptive = pp.adaptive_rho ? 1 : 0;
  dirty_[h] = 1;  // uploaded with the other new descriptors before the next launch
  *handle = h;
  return POGS_OK;
}

// Copy the descriptors added since the last upload to the device in one
// transfer (through a pinned mirror of the descriptor array).
int GroupEngine::flush_descriptors() {
  if (upload_pending_) {
    POGS_HIP_TRY(host_uploader().fence(s_));
    upload_pending_ = false;
  }
  int lo = cap_, hi = -1;
  for (int h = 0; h < cap_; ++h)
    if (dirty_[h]) {
      lo = std::min(lo, h);
      hi = h;
    }
  if (hi < 0) return POGS_OK;
  if (desc_copied_) POGS_HIP_TRY(hipEventSynchronize(desc_copied_));
  for (int h = lo; h <= hi; ++h)
    if (dirty_[h]) {
      probs_host_[h] = probs_[h];
      dirty_[h] = 0;
    }
  POGS_HIP_TRY(hipMemcpyAsync(probs_dev_ + lo, probs_host_ + lo, (size_t)(hi - lo + 1) * sizeof(GProb),
                              hipMemcpyHostToDevice, s_));
  if (!desc_copied_) POGS_HIP_TRY(hipEventCreateWithFlags(&desc_copied_, hipEventDisableTiming));
  POGS_HIP_TRY(hipEventRecord(desc_copied_, s_));
  return POGS_OK;
}

void GroupEngine::remove(int h) {
  if (h < 0 || h >= cap_ || !used_[h]) return;
  dirty_[h] = 0;
  if (upload_pending_) {  // a copy into this problem's memory may still run
    (void)host_uploader().fence(s_);
    upload_pending_ = false;
  }
  if (mem_[h].owned) {
    if (mem_[h].arena) (void)hipFreeAsync(mem_[h].arena, s_);
    if (mem_[h].ws) (void)hipFreeAsync(mem_[h].ws, s_);
  }
  mem_[h] = Mem{};
  used_[h] = 0;
}

// Concatenate the lists into the pinned staging buffer and one device
// buffer; ptrs[i] is the device address of list i.
int GroupEngine::upload_items(const std::vector<std::vector<GItem>> &lists, std::vector<const GItem *> *ptrs) {
  // the previous copy out of the pinned staging must have completed before
  // the staging is overwritten (the copy is asynchronous)
  if (items_copied_) POGS_HIP_TRY(hipEventSynchronize(items_copied_));
  size_t total = 0;
  for (const auto &l : lists) total += l.size();
  total = std::max<size_t>(total, 1);
  if (total > items_host_cap_) {
    if (items_host_) (void)hipHostFree(items_host_);
    items_host_ = nullptr;
    items_host_cap_ = 0;
    if (hipHostMalloc((void **)&items_host_, total * sizeof(GItem)) != hipSuccess) return POGS_ENOMEM;
    items_host_cap_ = total;
  }
  if (total > items_cap_) {
    if (items_dev_) (void)hipFreeAsync(items_dev_, s_);
    items_dev_ = nullptr;
    items_cap_ = 0;
    if (hipMallocAsync((void **)&items_dev_, total * sizeof(GItem), s_) != hipSuccess) return POGS_ENOMEM;
    items_cap_ = total;
  }
  ptrs->clear();
  size_t off = 0;
  for (const auto &l : lists) {
    if (!l.empty()) memcpy(items_host_ + off, l.data(), l.size() * sizeof(GItem));
    ptrs->push_back(items_dev_ + off);
    off += l.size();
  }
  if (off) {
    POGS_HIP_TRY(hipMemcpyAsync(items_dev_, items_host_, off * sizeof(GItem), hipMemcpyHostToDevice, s_));
    if (!items_copied_) POGS_HIP_TRY(hipEventCreateWithFlags(&items_copied_, hipEventDisableTiming));
    POGS_HIP_TRY(hipEventRecord(items_copied_, s_));
  }
  return POGS_OK;
}

int GroupEngine::refresh_status(const std::vector<int> &handles) {
  if (int rc0 = flush_descriptors()) return rc0;
  std::vector<std::vector<GItem>> lists(1);
  for (int h : handles) lists[0].push_back(GItem{h, 0, 0, 1, 1});
  std::vector<const GItem *> ptr;
  int rc;
  if ((rc = upload_items(lists, &ptr))) return rc;
  launch_group(G_GATHER, probs_dev_, ptr[0], (int)lists[0].size(), 0, s_);
  POGS_HIP_TRY(hipMemcpyAsync(status_host_, status_dev_, (size_t)cap_ * sizeof(GStatus), hipMemcpyDeviceToHost,
                              s_));
  POGS_HIP_TRY(hipStreamSynchronize(s_));
  POGS_HIP_TRY(hipGetLastError());
  return POGS_OK;
}

namespace {

// Problems in decreasing size, so the largest problems' items start first.
std::vector<int> by_size(const std::vector<GProb> &probs, const std::vector<int> &handles) {
  std::vector<int> hs(handles);
  std::stable_sort(hs.begin(), hs.end(), [&](int a, int b) {
    return (double)probs[a].it.m * probs[a].it.n > (double)probs[b].it.m * probs[b].it.n;
  });
  return hs;
}

void push_range(std::vector<GItem> &l, int h, int nx, int ny = 1) {
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) l.push_back(GItem{h, x, y, nx, ny});
}

}  // namespace

int GroupEngine::setup(const std::vector<int> &handles) {
  if (handles.empty()) return POGS_OK;
  if (int rc0 = flush_descriptors()) return rc0;
  const std::vector<int> hs = by_size(probs_, handles);
  enum { L_ROWS, L_TILES, L_NORM, L_SCALE, L_FN, L_GRAM, L_TRTRI, L_POTRF, L_KINV, L_INIT, L_FIXED };
  int max_eq = 0, max_nbt = 0;
  for (int h : hs) {
    max_eq = std::max(max_eq, probs_[h].equil_iters);
    max_nbt = std::max(max_nbt, probs_[h].nbt);
  }
  // lists: fixed ones, then per sweep 4 (by U) + colfinish, then per step panel + update
  std::vector<std::vector<GItem>> lists(L_FIXED + 5 * max_eq + 2 * max_nbt);
  auto sweep = [&](int it, int U) -> std::vector<GItem> & { return lists[L_FIXED + 5 * it + (U - 1)]; };
  auto colfin = [&](int it) -> std::vector<GItem> & { return lists[L_FIXED + 5 * it + 4]; };
  auto panel = [&](int kb) -> std::vector<GItem> & { return lists[L_FIXED + 5 * max_eq + 2 * kb]; };
  auto update = [&](int kb) -> std::vector<GItem> & { return lists[L_FIXED + 5 * max_eq + 2 * kb + 1]; };
  // Gram tiles: largest K range first
  std::vector<std::pair<double, GItem>> gram;
  for (int h : hs) {
    const GProb &P = probs_[h];
    const Geo g = geo(P.it.m, P.it.n);
    if (!P.colmajor) push_range(lists[L_ROWS], h, (int)cdiv(g.m, kLayRows));
    else push_range(lists[L_TILES], h, (int)cdiv(g.ld, 32), (int)cdiv(g.m, 32));
    for (int it = 0; it < P.equil_iters; ++it) {
      push_range(sweep(it, g.eq_U), h, g.eq_nsplit);
      push_range(colfin(it), h, g.n_dual);
    }
    push_range(lists[L_NORM], h, (int)cdiv(g.m + g.n, 256));
    push_range(lists[L_SCALE], h, (int)cdiv(g.n, 256), std::min(g.m, 32));
    for (int y = 0; y < 2; ++y) {
      const int len = y ? g.n : g.m;
      const int nb = (int)cdiv(len, kBlock);
      for (int x = 0; x < nb; ++x) lists[L_FN].push_back(GItem{h, x, y, nb, 2});
    }
    const double kdim = g.tall ? g.m : g.n;
    for (int t = 0; t < g.ntp; ++t) gram.push_back({kdim, GItem{h, t, 0, g.ntp, 1}});
    push_range(lists[L_TRTRI], h, (int)cdiv(g.Q, 32));
    push_range(lists[L_POTRF], h, 1);
    for (int kb = 0; kb < g.nbt; ++kb) {
      const int rest = g.nbt - kb - 1;
      push_range(panel(kb), h, rest + kb + 1);
      if (rest > 0) push_range(update(kb), h, rest * (rest + 1) / 2 + rest * (kb + 1));
    }
    push_range(lists[L_KINV], h, g.nbt * (g.nbt + 1) / 2);
    push_range(lists[L_INIT], h, 1);
  }
  std::stable_sort(gram.begin(), gram.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
  for (auto &pr : gram) lists[L_GRAM].push_back(pr.second);
  std::vector<const GItem *> ptr;
  int rc;
  if ((rc = upload_items(lists, &ptr))) return rc;
  auto go = [&](int phase, int li, int arg = 0) {
    launch_group(phase, probs_dev_, ptr[li], (int)lists[li].size(), arg, s_);
  };
  go(G_LAYOUT_ROWS, L_ROWS);
  go(G_LAYOUT_TILES, L_TILES);
  for (int it = 0; it < max_eq; ++it) {
    for (int U = 1; U <= 4; ++U) go(G_EQ_SWEEP, L_FIXED + 5 * it + (U - 1), U);
    go(G_EQ_COLFINISH, L_FIXED + 5 * it + 4);
  }
  go(G_EQ_NORMALIZE, L_NORM);
  go(G_SCALE_MATRIX, L_SCALE);
  go(G_SCALE_FN, L_FN);
  go(G_GRAM, L_GRAM);
  go(G_TRTRI_INIT, L_TRTRI);
  go(G_POTRF0, L_POTRF);
  for (int kb = 0; kb < max_nbt; ++kb) {
    go(G_PANEL, L_FIXED + 5 * max_eq + 2 * kb, kb);
    go(G_UPDATE, L_FIXED + 5 * max_eq + 2 * kb + 1, kb);
  }
  go(G_KINV, L_KINV);
  go(G_INIT_STATE, L_INIT);
  POGS_HIP_TRY(hipGetLastError());
  // the setup workspace goes back to the pool once the kernels above are done
  for (int h : hs) {
    if (mem_[h].ws && mem_[h].owned) (void)hipFreeAsync(mem_[h].ws, s_);
    mem_[h].ws = nullptr;
  }
  return refresh_status(handles);
}

int GroupEngine::run_chunk(const std::vector<int> &handles, int chunk) {
  if (handles.empty()) return POGS_OK;
  if (int rc0 = flush_descriptors()) return rc0;
  chunk += chunk & 1;  // even: the state after the chunk is in st[0]
  const std::vector<int> hs = by_size(probs_, handles);
  enum { PROX, P1T, P1W64, P1W16, FIN1, SOL64, SOL16, P2T64, P2T16, P2W, FIN2, PREV, NLIST };
  std::vector<std::vector<GItem>> lists(NLIST);
  for (int h : hs) {
    const GProb &P = probs_[h];
    const Geo g = geo(P.it.m, P.it.n);
    push_range(lists[PROX], h, g.nbx + g.nby);
    const int rows_a = (int)cdiv(g.m, g.lpr16 ? kGRows16 : kGRows64);
    const int rows_k = (int)cdiv(g.q, g.lpr16k ? kGRows16 : kGRows64);
    if (g.tall) {
      push_range(lists[P1T], h, g.tiles, g.splits);
      push_range(lists[FIN1], h, g.n_dual);
      push_range(lists[g.lpr16 ? P2T16 : P2T64], h, rows_a);
    } else {
      push_range(lists[g.lpr16 ? P1W16 : P1W64], h, rows_a);
      push_range(lists[P2W], h, g.tiles, g.splits);
      push_range(lists[FIN2], h, g.n_dual);
    }
    push_range(lists[g.lpr16k ? SOL16 : SOL64], h, rows_k);
    push_range(lists[PREV], h, 1);
  }
  std::vector<const GItem *> ptr;
  int rc;
  if ((rc = upload_items(lists, &ptr))) return rc;
  auto go = [&](int phase, int li, int par) {
    launch_group(phase, probs_dev_, ptr[li], (int)lists[li].size(), par, s_);
  };
  for (int i = 0; i < chunk; ++i) {
    const int par = i & 1;
    go(G_PROX, PROX, par);
    go(G_PASS1_T, P1T, par);
    go(G_PASS1_W64, P1W64, par);
    go(G_PASS1_W16, P1W16, par);
    go(G_FINISH1, FIN1, par);
    go(G_SOLVE64, SOL64, par);
    go(G_SOLVE16, SOL16, par);
    go(G_PASS2_T64, P2T64, par);
    go(G_PASS2_T16, P2T16, par);
    go(G_PASS2_W, P2W, par);
    go(G_FINISH2, FIN2, par);
  }
  go(G_PREVIEW, PREV, 1);
  POGS_HIP_TRY(hipGetLastError());
  return refresh_status(handles);
}

int GroupEngine::finish(const std::vector<int> &handles) {
  if (handles.empty()) return POGS_OK;
  if (int rc0 = flush_descriptors()) return rc0;
  std::vector<std::vector<GItem>> lists(1);
  for (int h : handles) {
    const GProb &P = probs_[h];
    push_range(lists[0], h, P.it.nbx + P.it.nby);
  }
  std::vector<const GItem *> ptr;
  int rc;
  if ((rc = upload_items(lists, &ptr))) return rc;
  launch_group(G_UNSCALE, probs_dev_, ptr[0], (int)lists[0].size(), 0, s_);
  POGS_HIP_TRY(hipGetLastError());
  return refresh_status(handles);
}

int GroupEngine::copy_out_many(const std::vector<int> &handles, const std::vector<pogs_result *> &outs) {
  // device destinations: direct copies; host destinations: every block into
  // one pinned buffer, one synchronisation, then to the callers' buffers
  size_t total = 0;
  for (size_t k = 0; k < handles.size(); ++k)
    if (outs[k]->mem != POGS_DEVICE) total += (size_t)2 * (m(handles[k]) + n(handles[k]));
  if (total * 4 > out_stage_cap_) {
    if (out_stage_) (void)hipHostFree(out_stage_);
    out_stage_ = nullptr;
    out_stage_cap_ = 0;
    const size_t want = std::max<size_t>(total * 4, 1 << 20);
    if (hipHostMalloc((void **)&out_stage_, want) != hipSuccess) return POGS_ENOMEM;
    out_stage_cap_ = want;
  }
  size_t off = 0;
  for (size_t k = 0; k < handles.size(); ++k) {
    const pogs_result &r = *outs[k];
    if (r.mem == POGS_DEVICE) {
      int rc = copy_out(handles[k], r.x, r.y, r.mu, r.nu, POGS_DEVICE);
      if (rc) return rc;
      continue;
    }
    const GProb &P = probs_[handles[k]];
    const size_t len = (size_t)2 * (P.it.m + P.it.n);
    POGS_HIP_TRY(hipMemcpyAsync(out_stage_ + off, P.out, len * 4, hipMemcpyDeviceToHost, s_));
    off += len;
  }
  POGS_HIP_TRY(hipStreamSynchronize(s_));
  off = 0;
  for (size_t k = 0; k < handles.size(); ++k) {
    const pogs_result &r = *outs[k];
    if (r.mem == POGS_DEVICE) continue;
    const int mm = m(handles[k]), nn = n(handles[k]);
    const float *o = out_stage_ + off;
    if (r.x) memcpy(r.x, o, (size_t)nn * 4);
    if (r.y) memcpy(r.y, o + nn, (size_t)mm * 4);
    if (r.mu) memcpy(r.mu, o + nn + mm, (size_t)nn * 4);
    if (r.nu) memcpy(r.nu, o + 2 * nn + mm, (size_t)mm * 4);
    off += (size_t)2 * (mm + nn);
  }
  return POGS_OK;
}

int GroupEngine::copy_out(int h, void *x, void *y, void *mu, void *nu, pogs_mem mem) {
  const GProb &P = probs_[h];
  const int m = P.it.m, n = P.it.n;
  const float *o = P.out;
  const hipMemcpyKind k = mem == POGS_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (mem == POGS_DEVICE) {
    if (x) POGS_HIP_TRY(hipMemcpyAsync(x, o, (size_t)n * 4, k, s_));
    if (y) POGS_HIP_TRY(hipMemcpyAsync(y, o + n, (size_t)m * 4, k, s_));
    if (mu) POGS_HIP_TRY(hipMemcpyAsync(mu, o + n + m, (size_t)n * 4, k, s_));
    if (nu) POGS_HIP_TRY(hipMemcpyAsync(nu, o + 2 * n + m, (size_t)m * 4, k, s_));
    return POGS_OK;
  }
  // one copy of the whole block into pinned memory, then to the caller
  const size_t bytes = (size_t)2 * (m + n) * 4;
  if (bytes > out_stage_cap_) {
    if (out_stage_) (void)hipHostFree(out_stage_);
    out_stage_ = nullptr;
    out_stage_cap_ = 0;
    if (hipHostMalloc((void **)&out_stage_, std::max<size_t>(bytes, 1 << 20)) != hipSuccess) return POGS_ENOMEM;
    out_stage_cap_ = std::max<size_t>(bytes, 1 << 20);
  }
  POGS_HIP_TRY(hipMemcpyAsync(out_stage_, o, bytes, hipMemcpyDeviceToHost, s_));
  POGS_HIP_TRY(hipStreamSynchronize(s_));
  if (x) memcpy(x, out_stage_, (size_t)n * 4);
  if (y) memcpy(y, out_stage_ + n, (size_t)m * 4);
  if (mu) memcpy(mu, out_stage_ + n + m, (size_t)n * 4);
  if (nu) memcpy(nu, out_stage_ + 2 * n + m, (size_t)m * 4);
  return POGS_OK;
}

}  // namespace pogs
