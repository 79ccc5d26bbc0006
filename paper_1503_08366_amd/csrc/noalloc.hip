// Allocation-free prox evaluation (the elementwise prox of Section 5's
// parametric form): the function's parameters are staged in `scratch`, a
// file-scope device array of POGS_NOALLOC_SCRATCH_BYTES that every GPU the
// library runs on holds until the process ends, instead of in memory allocated
// per call.  Host code never passes `scratch` itself to a kernel or a copy (in
// host code the name stands for a host-side shadow, not a device address): it
// looks up the array's device address once per device with
// hipGetSymbolAddress and uses that address everywhere.
//
// Layout of one call in scratch: the h codes (cnt bytes), then a, b, c, d, e
// as float64 (cnt entries each, only those the caller supplied), each piece at
// a 256-byte boundary; cnt = len (per-element parameters) or 1 (broadcast).
// The kernel converts each float64 parameter to the iteration type exactly
// as pogs_prox's host expansion does, so both entry points give the same bits.
#include <mutex>

#include "hostutil.hpp"

namespace pogs {
namespace {

constexpr size_t kScratchBytes = POGS_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices];  // device address of scratch, per device

// Device address of scratch on the current device (looked up on the first
// call on that device, with it current).
int scratch_address(unsigned char **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return POGS_EDEVICE;
  if (dev < 0 || dev >= kMaxDevices) return POGS_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      fprintf(stderr, "pogs: hipGetSymbolAddress(scratch) failed: %s\n", hipGetErrorString(e));
      return POGS_EDEVICE;
    }
    g_scratch_ptr[dev] = (unsigned char *)p;
  }
  *out = g_scratch_ptr[dev];
  return POGS_OK;
}

struct StagedFn {
  const uint8_t *h;
  const double *prm[5];  // a, b, c, d, e; NULL = default
  int stride;            // 1 per element, 0 broadcast entry 0
};

template <typename T>
__global__ __launch_bounds__(kBlock) void prox_staged_kernel(StagedFn f, T rho, const T *__restrict__ v,
                                                             T *__restrict__ out, int len) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= len) return;
  const int k = f.stride ? i : 0;
  const T a = f.prm[0] ? (T)f.prm[0][k] : T(1);
  const T b = f.prm[1] ? (T)f.prm[1][k] : T(0);
  const T c = f.prm[2] ? (T)f.prm[2][k] : T(1);
  const T d = f.prm[3] ? (T)f.prm[3][k] : T(0);
  const T e = f.prm[4] ? (T)f.prm[4][k] : T(0);
  out[i] = prox_param<T>(f.h[k], a, b, c, d, e, v[i], rho);
}

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace
}  // namespace pogs

using namespace pogs;

extern "C" int pogs_prox_noalloc(const pogs_fn *fn, pogs_dtype dt, double rho, const void *v, void *out,
                                 void *stream) {
  if (!fn || !v || !out || !(rho > 0.0) || !std::isfinite(rho)) return POGS_EINVAL;
  if (dt != POGS_F32 && dt != POGS_F64) return POGS_EINVAL;
  if (fn->len <= 0 || fn->len > (int64_t)INT32_MAX) return POGS_EINVAL;
  int rc;
  if ((rc = check_fn(fn, fn->len))) return rc;
  const size_t cnt = fn->stride ? (size_t)fn->len : 1;
  const double *src[5] = {fn->a, fn->b, fn->c, fn->d, fn->e};
  size_t need = round256(cnt);
  for (int j = 0; j < 5; ++j)
    if (src[j]) need += round256(cnt * 8);
  if (need > kScratchBytes) return POGS_ETOOBIG;
  unsigned char *base = nullptr;
  if ((rc = scratch_address(&base))) return rc;
  hipStream_t s = (hipStream_t)stream;
  StagedFn f{};
  f.stride = fn->stride ? 1 : 0;
  size_t off = 0;
  POGS_HIP_TRY(hipMemcpyAsync(base, fn->h, cnt, hipMemcpyHostToDevice, s));
  f.h = base;
  off = round256(cnt);
  for (int j = 0; j < 5; ++j) {
    if (!src[j]) continue;
    POGS_HIP_TRY(hipMemcpyAsync(base + off, src[j], cnt * 8, hipMemcpyHostToDevice, s));
    f.prm[j] = (const double *)(base + off);
    off += round256(cnt * 8);
  }
  const int len = (int)fn->len;
  if (dt == POGS_F32)
    hipLaunchKernelGGL(prox_staged_kernel<float>, dim3(cdiv(len, kBlock)), dim3(kBlock), 0, s, f, (float)rho,
                       (const float *)v, (float *)out, len);
  else
    hipLaunchKernelGGL(prox_staged_kernel<double>, dim3(cdiv(len, kBlock)), dim3(kBlock), 0, s, f, rho,
                       (const double *)v, (double *)out, len);
  POGS_HIP_TRY(hipGetLastError());
  POGS_HIP_TRY(hipStreamSynchronize(s));
  return POGS_OK;
}
