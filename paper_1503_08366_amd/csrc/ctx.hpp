// The context object behind pogs_ctx (shared by the C ABI translation units).
#pragma once

#include <algorithm>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace pogs {

// Blocks of contexts that were freed after their stream had drained, kept
// for the next allocation of the same size on the same device: a context
// created after another one of the same shape takes its blocks back without
// a call into the stream-ordered pool (each hipFreeAsync costs the host
// 7-45 us there, measured on MI355X).  At most kKeep bytes are kept per
// process; past that the oldest go back to the pool.
class SpareBlocks {
 public:
  static constexpr size_t kKeep = 4ull << 30;
  void *take(int dev, size_t bytes) {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto it = blocks_.begin(); it != blocks_.end(); ++it)
      if (it->dev == dev && it->bytes == bytes) {
        void *p = it->ptr;
        held_ -= bytes;
        blocks_.erase(it);
        return p;
      }
    return nullptr;
  }
  // p is idle (no queued work uses it); s orders the frees of evicted blocks
  void keep(int dev, void *p, size_t bytes, hipStream_t s) {
    std::lock_guard<std::mutex> lk(mu_);
    blocks_.push_back({dev, p, bytes});
    held_ += bytes;
    while (held_ > kKeep && !blocks_.empty()) {
      (void)hipFreeAsync(blocks_.front().ptr, s);
      held_ -= blocks_.front().bytes;
      blocks_.erase(blocks_.begin());
    }
  }
  // every kept block of device dev back to the pool (before retrying an
  // allocation that failed)
  bool flush(int dev, hipStream_t s) {
    std::lock_guard<std::mutex> lk(mu_);
    bool any = false;
    for (auto it = blocks_.begin(); it != blocks_.end();) {
      if (it->dev == dev) {
        (void)hipFreeAsync(it->ptr, s);
        held_ -= it->bytes;
        it = blocks_.erase(it);
        any = true;
      } else {
        ++it;
      }
    }
    return any;
  }

 private:
  struct Block {
    int dev;
    void *ptr;
    size_t bytes;
  };
  std::mutex mu_;
  std::vector<Block> blocks_;
  size_t held_ = 0;
};
inline SpareBlocks &spare_blocks() {
  static SpareBlocks s;
  return s;
}

// Device allocations owned by a context, freed together.  Allocation is
// stream-ordered (hipMallocAsync / hipFreeAsync on the stream that uses the
// memory) from the device's default pool, which keeps freed memory cached up
// to a threshold: a context created after another one reuses its memory
// without a device synchronisation or an operating-system call.  Blocks
// released while the stream is known to be idle go to spare_blocks().
struct DevArena {
  hipStream_t stream = nullptr;
  struct Held {
    void *ptr;
    size_t bytes;
  };
  std::vector<Held> ptrs;
  int dev = -1;
  explicit DevArena(hipStream_t s = nullptr) : stream(s) { configure_pool(); }
  DevArena(const DevArena &) = delete;
  DevArena &operator=(const DevArena &) = delete;
  int alloc(void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0) bytes = 16;
    if (dev < 0 && hipGetDevice(&dev) != hipSuccess) return POGS_EDEVICE;
    *p = spare_blocks().take(dev, bytes);
    if (!*p && hipMallocAsync(p, bytes, stream) != hipSuccess) {
      *p = nullptr;
      (void)hipGetLastError();
      if (!spare_blocks().flush(dev, stream) || hipMallocAsync(p, bytes, stream) != hipSuccess) {
        *p = nullptr;
        return POGS_ENOMEM;
      }
    }
    ptrs.push_back({*p, bytes});
    return POGS_OK;
  }
  void release(void *p) {
    auto it = std::find_if(ptrs.begin(), ptrs.end(), [p](const Held &h) { return h.ptr == p; });
    if (it != ptrs.end()) {
      (void)hipFreeAsync(it->ptr, stream);
      ptrs.erase(it);
    }
  }
  // Last allocated first: freeing a large block ahead of smaller ones made
  // the next free take 0.3-1.2 ms in the stream-ordered pool (measured on
  // MI355X); in reverse order every free takes tens of microseconds.  idle:
  // the caller has drained the stream, so the blocks may be kept for reuse.
  void free_all(bool idle = false) {
    for (auto it = ptrs.rbegin(); it != ptrs.rend(); ++it) {
      if (idle) spare_blocks().keep(dev, it->ptr, it->bytes, stream);
      else (void)hipFreeAsync(it->ptr, stream);
    }
    ptrs.clear();
  }
  ~DevArena() { free_all(); }

  // Keep up to kPoolKeep bytes of freed memory cached in the current
  // device's default pool (once per device).
  static void configure_pool() {
    static std::mutex mu;
    static std::vector<int> done;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(mu);
    if (std::find(done.begin(), done.end(), dev) != done.end()) return;
    done.push_back(dev);
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) != hipSuccess) return;
    uint64_t keep = kPoolKeep;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  static constexpr uint64_t kPoolKeep = 16ull << 30;
};

// Small pinned host blocks (control-block read-backs), carved from pinned
// pages that live until the process ends: pinning costs far more than a
// small solve's host work.
class PinnedSlab {
 public:
  static constexpr size_t kChunk = 1024, kPage = 64 * 1024;
  void *get() {
    std::lock_guard<std::mutex> lk(mu_);
    if (free_.empty()) {
      void *pg = nullptr;
      if (hipHostMalloc(&pg, kPage) != hipSuccess) return nullptr;
      for (size_t i = 0; i < kPage / kChunk; ++i) free_.push_back((char *)pg + i * kChunk);
    }
    void *p = free_.back();
    free_.pop_back();
    return p;
  }
  void put(void *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu_);
    free_.push_back(p);
  }

 private:
  std::mutex mu_;
  std::vector<void *> free_;
};
inline PinnedSlab &pinned_slab() {
  static PinnedSlab s;
  return s;
}

// A grow-only pinned staging buffer for host-to-device uploads, one user at
// a time: acquire() waits until the previous user's copy has completed,
// release(stream) marks the end of this user's copies on its stream.
class PinnedStage {
 public:
  void *acquire(size_t bytes) {
    mu_.lock();
    if (ev_) (void)hipEventSynchronize(ev_);
    if (bytes > cap_) {
      if (buf_) (void)hipHostFree(buf_);
      buf_ = nullptr;
      cap_ = 0;
      const size_t want = std::max<size_t>(bytes, 1 << 20);
      if (hipHostMalloc(&buf_, want) != hipSuccess) {
        buf_ = nullptr;
        mu_.unlock();
        return nullptr;
      }
      cap_ = want;
    }
    return buf_;
  }
  void release(hipStream_t s) {
    if (!ev_) (void)hipEventCreateWithFlags(&ev_, hipEventDisableTiming);
    if (ev_) (void)hipEventRecord(ev_, s);
    mu_.unlock();
  }

 private:
  std::mutex mu_;
  void *buf_ = nullptr;
  size_t cap_ = 0;
  hipEvent_t ev_ = nullptr;
};
inline PinnedStage &pinned_stage() {
  static PinnedStage s;
  return s;
}

// Sub-buffers of one allocation, each aligned to 256 bytes: first pass
// records offsets, then base() turns them into pointers.
struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    off = (size_t)round_up((int64_t)off, 256);
    const size_t o = off;
    off += std::max<size_t>(bytes, 1);
    return o;
  }
};

}  // namespace pogs

using namespace pogs;

// ---------------------------------------------------------------------------
// Context
// ---------------------------------------------------------------------------
struct pogs_ctx {
  int64_t m = 0, n = 0;
  int ld = 0, q = 0, Q = 0, ldk = 0;
  pogs_dtype dt = POGS_F32;
  pogs_params params{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  DevArena arena;
  void *A = nullptr;     // scaled matrix, T
  void *Kinv = nullptr;  // (I + G)^{-1}, T (direct projection only)
  int proj = POGS_PROJ_DIRECT;  // projection the context was set up for
  // sparse contexts: A^ and A^T in compressed rows (int32 indices, T values)
  bool sparse = false;
  int64_t nnz = 0;
  int *sp_rp = nullptr, *sp_ci = nullptr, *sp_rpt = nullptr, *sp_cit = nullptr;
  void *sp_va = nullptr, *sp_vat = nullptr;
  int sp_lpr = 0, sp_grid = 0, sp_lprt = 0, sp_gridt = 0;
  int sp_nseg = 1;  // column segments of the A^T copy
  void *sp_pair = nullptr;  // 2 m entries of T
  double *D = nullptr, *E = nullptr;
  // iteration state (T): x y xt yt xh yh mu nu cx dy rhs, outputs xo yo muo nuo
  void *vec = nullptr;
  // scaled functions (T) and original functions (float64)
  uint8_t *fh = nullptr, *gh = nullptr, *fh0 = nullptr, *gh0 = nullptr;
  void *fs = nullptr, *gs = nullptr;     // 5 arrays each, T
  double *f0 = nullptr, *g0 = nullptr;   // 5 arrays each, float64
  // fh0 | gh0 | f0 | g0 form one block (fn_raw, fn_bytes) uploaded in one copy
  void *fn_raw = nullptr;
  size_t fn_bytes = 0, off_gh0 = 0, off_f0 = 0, off_g0 = 0;
  double *part = nullptr, *slots = nullptr;
  unsigned *counters = nullptr;
  Ctrl *ctrl = nullptr;
  Ctrl *ctrl_host = nullptr;   // pinned
  double *obj_host = nullptr;  // pinned
  double *obj_dev = nullptr;
  int splits = 0, rps = 0, ncolp = 0;
  int nbx = 0, nby = 0, n_pri = 0, n_dual = 0;
  int smu_cap = 0, syh_cap = 0;  // s_mu / s_yh slots per parity: max(nbx, n_dual), max(nby, splits, fp_blocks)
  int fp_blocks = 0;   // workgroups of the one-pass kernel (0: the context cannot run it)
  bool fused = false;  // iterations run the one-pass tall launches (set per solve, see IterArgs::fused)
  double ms_setup = 0.0;
  hipGraphExec_t graph = nullptr;
  unsigned *flags_host = nullptr;  // setup flags read back by pogs_init (pinned)
  int graph_chunk = 0;
  int graph_cg_cap = 0;  // CGLS step cap of the captured graph (0: direct projection)
  int graph_gap = 0;     // the captured graph runs the gap test
  int nt_rows = 0, nt_cols = 0;  // load policy of the passes over A (size rule or autotuned)
  bool solved = false;  // functions uploaded by a previous solve

  size_t esz() const { return dt == POGS_F32 ? 4 : 8; }
  template <typename T> T *vecp(int idx) const {
    // vectors 0..3: x, y, xt, yt; 4..7: xh, yh, mu, nu; 8: cx, 9: dy, 10: rhs; 11..14: outputs;
    // 15..17: CGLS p, q, s; 18..23: the second half-step set xh, yh, mu, nu, cx, dy (odd
    // iterations of the one-pass iteration)
    static const int kind[24] = {0, 1, 0, 1, 0, 1, 0, 1, 0, 1, 2, 0, 1, 0, 1, 0, 1, 0,
                                 0, 1, 0, 1, 0, 1};  // 0: n, 1: m, 2: q
    size_t off = 0;
    const size_t L[3] = {(size_t)round_up(n, 64), (size_t)round_up(m, 64), (size_t)round_up(q, 64)};
    for (int i = 0; i < idx; ++i) off += L[kind[i]];
    return reinterpret_cast<T *>(vec) + off;
  }
  size_t vec_elems() const {  // the 24 vectors of vecp: 12 of length n, 11 of m, 1 of q
    return 12 * (size_t)round_up(n, 64) + 11 * (size_t)round_up(m, 64) + (size_t)round_up(q, 64);
  }
  // The arguments of iteration parity `set`: the one-pass iteration keeps the
  // half step of even iterations in vectors 4..9 and of odd ones in 18..23
  // (iteration k computes part of iteration k + 1's half step while its own is
  // still needed); every other mode uses set 0.
  template <typename T> IterArgs<T> iter_args(int set = 0) const {
    IterArgs<T> p{};
    p.m = (int)m;
    p.n = (int)n;
    p.ld = ld;
    p.q = q;
    p.ldk = ldk;
    p.A = (const T *)A;
    p.Kinv = (const T *)Kinv;
    const T *fsp = (const T *)fs;
    const T *gsp = (const T *)gs;
    p.f = FnDev<T>{fh, fsp, fsp + m, fsp + 2 * m, fsp + 3 * m, fsp + 4 * m};
    p.g = FnDev<T>{gh, gsp, gsp + n, gsp + 2 * n, gsp + 3 * n, gsp + 4 * n};
    p.x = vecp<T>(0);
    p.y = vecp<T>(1);
    p.xt = vecp<T>(2);
    p.yt = vecp<T>(3);
    p.xh = vecp<T>(4);
    p.yh = vecp<T>(5);
    p.mu = vecp<T>(6);
    p.nu = vecp<T>(7);
    p.cx = vecp<T>(8);
    p.dy = vecp<T>(9);
    p.rhs = vecp<T>(10);
    {
      T *h0[6] = {vecp<T>(4), vecp<T>(5), vecp<T>(6), vecp<T>(7), vecp<T>(8), vecp<T>(9)};
      T *h1[6] = {vecp<T>(18), vecp<T>(19), vecp<T>(20), vecp<T>(21), vecp<T>(22), vecp<T>(23)};
      T **cur = set ? h1 : h0, **nxt = set ? h0 : h1;
      p.xh = cur[0];
      p.yh = cur[1];
      p.mu = cur[2];
      p.nu = cur[3];
      p.cx = cur[4];
      p.dy = cur[5];
      p.nyh = nxt[1];
      p.nnu = nxt[3];
      p.ndy = nxt[5];
    }
    p.part = part;
    p.nbx = nbx;
    p.nby = nby;
    p.fused = fused ? 1 : 0;
    p.n_smu = fused ? n_dual : nbx;
    p.n_syh = fused ? std::max(splits, fp_blocks) : nby;
    p.s_mu = slots;                    // 2 x n_smu (by iteration parity), room for 2 x smu_cap
    p.s_yh = slots + 2 * smu_cap;      // 2 x n_syh, room for 2 x syh_cap
    p.s_pri = p.s_yh + 2 * syh_cap;    // n_pri, room for max(n_pri, fp_blocks)
    p.s_dual = p.s_pri + std::max(n_pri, fp_blocks);
    p.par = 0;
    p.n_pri = fused ? fp_blocks : n_pri;
    p.fp_blocks = fp_blocks;
    p.n_dual = n_dual;
    p.ctrl = ctrl;
    p.nt_rows = nt_rows;
    p.nt_cols = nt_cols;
    p.pv = vecp<T>(15);
    p.qv = vecp<T>(16);
    p.sv = vecp<T>(17);
    p.s_gam = p.s_dual + n_dual;     // 2 x n_dual
    p.s_sig = p.s_gam + 2 * n_dual;  // 2 x n_dual
    p.s_qq = p.s_sig + 2 * n_dual;   // n_pri
    p.s_gobj = p.s_qq + n_pri;       // nbx + nby
    p.s_gconj = p.s_gobj + nbx + nby;  // nbx + nby
    if (sparse) {
      p.sa = Csr<T>{sp_rp, sp_ci, (T *)sp_va, (int)m, sp_lpr, sp_grid, 1};
      p.sat = Csr<T>{sp_rpt, sp_cit, (T *)sp_vat, (int)n, sp_lprt, sp_gridt, sp_nseg};
      p.pair = (T *)sp_pair;
    }
    return p;
  }
  ~pogs_ctx() {
    if (graph) (void)hipGraphExecDestroy(graph);
    // device memory goes back to the pool in the order of the context's
    // stream (a caller's stream needs no wait: later work on it is ordered
    // after the frees, and the pool orders reuse on other streams); a stream
    // of the context's own is drained before it is destroyed
    arena.free_all();
    if (own_stream && stream) {
      (void)hipStreamSynchronize(stream);
      (void)hipStreamDestroy(stream);
    }
    pinned_slab().put(ctrl_host);
    pinned_slab().put(obj_host);
    pinned_slab().put(flags_host);
  }
};

