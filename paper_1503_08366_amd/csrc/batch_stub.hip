// Placeholder entry points for the lambda-path and batch engine (replaced by
// their implementations).
#include "internal.hpp"

extern "C" {
int pogs_solve_path(pogs_ctx *, int32_t, const pogs_fn *, const pogs_fn *, const pogs_params *, pogs_result *) {
  return POGS_EUNSUPPORTED;
}
int pogs_batch_create(pogs_batch **out, const pogs_batch_cfg *) {
  if (out) *out = nullptr;
  return POGS_EUNSUPPORTED;
}
int pogs_batch_submit(pogs_batch *, const pogs_problem *, uint64_t *) { return POGS_EUNSUPPORTED; }
int pogs_batch_poll(pogs_batch *, uint64_t, pogs_result *) { return POGS_EUNSUPPORTED; }
int pogs_batch_wait_all(pogs_batch *) { return POGS_EUNSUPPORTED; }
int pogs_batch_cancel(pogs_batch *, uint64_t) { return POGS_EUNSUPPORTED; }
int pogs_batch_destroy(pogs_batch *) { return POGS_OK; }
int pogs_solve_batch(int32_t, const pogs_problem *, pogs_result *, void *) { return POGS_EUNSUPPORTED; }
}
