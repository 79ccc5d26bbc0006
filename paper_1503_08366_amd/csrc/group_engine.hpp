// Host side of the grouped launches: per-problem device memory, work lists,
// the setup sequence and chunks of iterations over a set of resident
// problems.  Used by the one-call batch entry point and the serving engine.
#pragma once

#include <vector>

#include "group.hpp"
#include "hostutil.hpp"

namespace pogs {

class GroupEngine {
 public:
  // A validated problem.  A, f and g must stay valid until setup() of this
  // problem has returned.
  struct Input {
    int m = 0, n = 0;
    const float *A = nullptr;  // row-major (lda >= n) or column-major (lda >= m)
    bool colmajor = false;
    long long lda = 0;
    const HostFn *f = nullptr, *g = nullptr;
    pogs_params params{};
    // optional caller-owned device memory (split_bytes sizes; arena zeroed);
    // NULL: the engine allocates and frees its own.  Caller-provided
    // memory must be ready for the host uploader (host_uploader().order()
    // on the engine's stream after it was allocated and cleared).
    void *arena = nullptr, *ws = nullptr;
  };

  // Largest problems the grouped path takes: n and min(m, n) up to 4096.
  static bool fits(int m, int n);
  // Device bytes a problem holds while resident (persistent + setup workspace).
  static size_t bytes_for(int m, int n);
  // The same split into the persistent part and the setup workspace.
  static void split_bytes(int m, int n, size_t *arena, size_t *ws);

  GroupEngine(hipStream_t s, int capacity);
  ~GroupEngine();
  GroupEngine(const GroupEngine &) = delete;
  GroupEngine &operator=(const GroupEngine &) = delete;
  int init();  // device arrays; POGS_OK or an error

  // Allocate and upload one problem; *handle identifies it.
  int add(const Input &in, int *handle);
  // Run the setup (layout .. K^{-1}, initial state) of these problems.
  int setup(const std::vector<int> &handles);
  // Run `chunk` iterations (even) of these problems, then refresh their
  // status (status(h) afterwards).
  int run_chunk(const std::vector<int> &handles, int chunk);
  // Return to the original variables (objective in status(h).obj).
  int finish(const std::vector<int> &handles);
  // Copy x (n), y (m), mu (n), nu (m) of a finished problem to host or device
  // buffers (NULL skips); mem says where the buffers are.
  int copy_out(int handle, void *x, void *y, void *mu, void *nu, pogs_mem mem);
  // The same for several finished problems into outs[k]'s buffers (out->mem
  // says where), with one synchronisation for all host destinations.
  int copy_out_many(const std::vector<int> &handles, const std::vector<pogs_result *> &outs);
  void remove(int handle);

  const GStatus &status(int handle) const { return status_host_[handle]; }
  int m(int handle) const { return probs_[handle].it.m; }
  int n(int handle) const { return probs_[handle].it.n; }

 private:
  struct Mem {
    void *arena = nullptr;  // persistent
    void *ws = nullptr;     // setup workspace
    bool owned = false;     // allocated by the engine
  };
  int upload_items(const std::vector<std::vector<GItem>> &lists, std::vector<const GItem *> *ptrs);
  int flush_descriptors();
  int refresh_status(const std::vector<int> &handles);

  hipStream_t s_;
  int cap_;
  std::vector<GProb> probs_;        // host copies of the descriptors
  std::vector<Mem> mem_;
  std::vector<char> used_;
  std::vector<char> dirty_;         // descriptors not yet on the device
  GProb *probs_host_ = nullptr;     // pinned mirror of the descriptors
  hipEvent_t desc_copied_ = nullptr;  // the last copy out of probs_host_
  bool upload_pending_ = false;       // matrices uploaded without a fence on s_
  GProb *probs_dev_ = nullptr;
  GStatus *status_dev_ = nullptr;
  GStatus *status_host_ = nullptr;  // pinned
  GItem *items_dev_ = nullptr;
  size_t items_cap_ = 0;
  GItem *items_host_ = nullptr;     // pinned staging of the work lists
  size_t items_host_cap_ = 0;
  hipEvent_t items_copied_ = nullptr;  // the last copy out of items_host_
  char *fn_stage_ = nullptr;        // pinned ring staging the function parameters
  size_t fn_stage_cap_ = 0;
  size_t fn_stage_pos_ = 0;
  hipEvent_t fn_stage_event_ = nullptr;  // the last copy out of the ring
  float *out_stage_ = nullptr;      // pinned staging of returned vectors
  size_t out_stage_cap_ = 0;
};

}  // namespace pogs
