// Host-to-device uploads of large buffers in pageable memory.  A copy from
// pageable memory goes through the runtime's own staging, one host thread,
// at about half the PCIe rate (measured on MI355X: 27 GB/s pageable, 58 GB/s
// from pinned memory, 80 GB/s for a host memcpy on four threads).  Here the
// source is copied into a ring of pinned chunks by a small pool of threads
// while the DMA of the previous chunk runs (53+ GB/s).
//
// upload() and upload_rows() return once every byte has left the source
// (the caller may then reuse or free it, as after a pageable
// hipMemcpyAsync); the copies run on the uploader's own stream and the
// caller's stream waits for them.  Successive small uploads share a slot of
// the ring.  Calls are serialised
// (they share the link).  The ring and the threads live until the process
// ends (the pool is never destroyed: its threads wait on it).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>

namespace pogs {

// fn(p) for p in [0, parts), spread over the pool's threads and the caller;
// returns when every part has finished.  Runs from several threads take
// turns.
class CopyPool {
 public:
  explicit CopyPool(int workers) {
    for (int i = 0; i < workers; ++i) std::thread([this] { worker(); }).detach();
  }
  void run(int parts, const std::function<void(int)> &fn) {
    std::lock_guard<std::mutex> one(run_mu_);  // callers on several threads take turns
    std::unique_lock<std::mutex> lk(mu_);
    fn_ = &fn;
    parts_ = parts;
    next_ = 0;
    left_ = parts;
    cv_.notify_all();
    while (next_ < parts_) {
      const int p = next_++;
      lk.unlock();
      fn(p);
      lk.lock();
      --left_;
    }
    done_.wait(lk, [&] { return left_ == 0; });
    fn_ = nullptr;
  }

 private:
  void worker() {
    std::unique_lock<std::mutex> lk(mu_);
    for (;;) {
      cv_.wait(lk, [&] { return fn_ != nullptr && next_ < parts_; });
      const int p = next_++;
      const std::function<void(int)> *f = fn_;
      lk.unlock();
      (*f)(p);
      lk.lock();
      if (--left_ == 0) done_.notify_all();
    }
  }
  std::mutex run_mu_, mu_;
  std::condition_variable cv_, done_;
  const std::function<void(int)> *fn_ = nullptr;
  int parts_ = 0, next_ = 0, left_ = 0;
};

class HostUploader {
 public:
  static constexpr size_t kChunk = (size_t)16 << 20;   // ring slot
  static constexpr int kSlots = 4, kParts = 4;
  static constexpr size_t kDirect = (size_t)64 << 10;  // smaller copies go straight
  static constexpr size_t kParallel = (size_t)2 << 20; // pieces copied by the pool from here up

  // dst (device) <- src (host, bytes contiguous)
  hipError_t upload(void *dst, const void *src, size_t bytes, hipStream_t s) {
    return upload_rows(dst, src, bytes, bytes, 1, s);
  }

  // Later uploads start after the work queued on s so far (for uploads made
  // with order = false into memory that s made ready).
  hipError_t order(hipStream_t s) {
    std::lock_guard<std::mutex> lk(mu_);
    hipError_t e = setup();
    if (e != hipSuccess) return e;
    return (e = hipEventRecord(start_, s)) != hipSuccess ? e : hipStreamWaitEvent(us_, start_, 0);
  }

  // The caller's stream waits for every upload issued so far (for uploads
  // made with fence = false).
  hipError_t fence(hipStream_t s) {
    std::lock_guard<std::mutex> lk(mu_);
    if (!us_) return hipSuccess;
    hipError_t e = hipEventRecord(done_, us_);
    return e != hipSuccess ? e : hipStreamWaitEvent(s, done_, 0);
  }

  // dst (device, rows packed: rows x width bytes) <- rows of width bytes at
  // src + r * pitch (host).  Pitched rows wider than a slot use the
  // runtime's 2D copy.  fence = false: s does not wait for the copies; the
  // caller calls fence(s) before work of s reads or frees dst.  order =
  // false: the copies do not wait for the work queued on s; the caller has
  // called order(s) since dst became ready.  (A caller uploading many
  // buffers so keeps the copies back to back.)
  hipError_t upload_rows(void *dst, const void *src, size_t width, size_t pitch, size_t rows, hipStream_t s,
                         bool fence = true, bool order = true) {
    const size_t total = width * rows;
    const bool contiguous = rows == 1 || pitch == width;
    if (total < kDirect || (!contiguous && width > kChunk)) {
      if (contiguous) return hipMemcpyAsync(dst, src, total, hipMemcpyHostToDevice, s);
      return hipMemcpy2DAsync(dst, width, src, pitch, width, rows, hipMemcpyHostToDevice, s);
    }
    std::lock_guard<std::mutex> lk(mu_);
    hipError_t e = setup();
    if (e != hipSuccess) return e;
    // the copies run on the uploader's own stream, after the caller's prior
    // work (dst may be stream-ordered memory of the caller's stream), and the
    // caller's stream waits for them; no event of the ring is ever recorded
    // on a stream the uploader does not own
    if (order &&
        ((e = hipEventRecord(start_, s)) != hipSuccess || (e = hipStreamWaitEvent(us_, start_, 0)) != hipSuccess))
      return e;
    const char *from = (const char *)src;
    // contiguous: a piece is up to a slot of bytes; pitched: whole rows
    const size_t unit = contiguous ? 1 : width, step = contiguous ? 1 : pitch;
    const size_t count = contiguous ? total : rows, per_piece = contiguous ? kChunk : kChunk / width;
    for (size_t done = 0; done < count;) {
      const size_t nu = std::min(per_piece, count - done), len = nu * unit;
      char *stage;
      if ((e = take(len, &stage)) != hipSuccess) return e;
      const size_t parts = len >= kParallel ? kParts : 1;
      auto copy = [&](int p) {
        const size_t lo = nu * p / parts, hi = nu * (p + 1) / parts;
        if (contiguous) std::memcpy(stage + lo, from + done + lo, hi - lo);
        else
          for (size_t r = lo; r < hi; ++r) std::memcpy(stage + r * width, from + (done + r) * step, width);
      };
      if (parts > 1) pool_->run((int)parts, copy);
      else copy(0);
      if ((e = hipMemcpyAsync((char *)dst + done * unit, stage, len, hipMemcpyHostToDevice, us_)) != hipSuccess)
        return e;
      if ((e = hipEventRecord(slot_[cur_].ev, us_)) != hipSuccess) return e;
      done += nu;
    }
    if (!fence) return hipSuccess;
    if ((e = hipEventRecord(done_, us_)) != hipSuccess) return e;
    return hipStreamWaitEvent(s, done_, 0);
  }

 private:
  // Space for len bytes in the current slot, or the next one once the
  // current is full; a slot is reused after its event (recorded after the
  // last copy out of it).
  hipError_t take(size_t len, char **out) {
    Slot *sl = &slot_[cur_];
    if (sl->fill + len > kChunk) {
      cur_ = (cur_ + 1) % kSlots;
      sl = &slot_[cur_];
      if (sl->fill) {
        const hipError_t e = hipEventSynchronize(sl->ev);
        if (e != hipSuccess) return e;
      }
      sl->fill = 0;
    }
    *out = ring_ + (size_t)cur_ * kChunk + sl->fill;
    sl->fill += (len + 255) / 256 * 256;
    return hipSuccess;
  }
  hipError_t setup() {
    if (ring_) return hipSuccess;
    hipError_t e;
    for (int i = 0; i < kSlots; ++i)
      if (!slot_[i].ev && (e = hipEventCreateWithFlags(&slot_[i].ev, hipEventDisableTiming)) != hipSuccess) return e;
    if (!start_ && (e = hipEventCreateWithFlags(&start_, hipEventDisableTiming)) != hipSuccess) return e;
    if (!done_ && (e = hipEventCreateWithFlags(&done_, hipEventDisableTiming)) != hipSuccess) return e;
    if (!us_ && (e = hipStreamCreateWithFlags(&us_, hipStreamNonBlocking)) != hipSuccess) return e;
    if (!pool_) pool_ = new CopyPool(kParts - 1);
    char *r = nullptr;
    if ((e = hipHostMalloc((void **)&r, kChunk * kSlots, hipHostMallocDefault)) != hipSuccess) return e;
    ring_ = r;
    return hipSuccess;
  }
  struct Slot {
    hipEvent_t ev = nullptr;
    size_t fill = 0;
  };
  std::mutex mu_;
  char *ring_ = nullptr;
  Slot slot_[kSlots];
  int cur_ = 0;
  hipStream_t us_ = nullptr;
  hipEvent_t start_ = nullptr, done_ = nullptr;
  CopyPool *pool_ = nullptr;
};

// A pool for other host-side copies (the serving engine's private copy of
// each request), separate from the uploader's so the two run side by side.
inline CopyPool &host_pool() {
  static CopyPool *p = new CopyPool(3);
  return *p;
}

// One uploader per process (never destroyed: its threads and pinned ring
// outlive every context).
inline HostUploader &host_uploader() {
  static HostUploader *u = new HostUploader();
  return *u;
}

}  // namespace pogs
