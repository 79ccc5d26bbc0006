// Host-side argument checks and expansion shared by the C ABI entry points.
#pragma once

#include <cmath>
#include <vector>

#include "internal.hpp"
#include "prox.hpp"

namespace pogs {

inline bool finite(double v) { return std::isfinite(v); }

// Expand a pogs_fn into per-element float64 arrays (host); validate it.
struct HostFn {
  std::vector<uint8_t> h;
  std::vector<double> a, b, c, d, e;
};

// One entry of a separable function: a known h code, finite parameters,
// c >= 0 and e >= 0 (convexity, Section 5), a != 0 where c > 0 (else the h
// term would be constant).
inline bool fn_entry_ok(uint8_t h, double a, double b, double c, double d, double e) {
  return h < kNumH && finite(a) && finite(b) && finite(c) && finite(d) && finite(e) && c >= 0.0 && e >= 0.0 &&
         !(c > 0.0 && a == 0.0);
}

// Validate a pogs_fn of length len in place (no copies): known h codes,
// finite parameters, c >= 0 and e >= 0 (convexity), a != 0 where c > 0.
inline int check_fn(const pogs_fn *fn, int64_t len) {
  if (!fn || fn->len != len || len <= 0 || !fn->h || (fn->stride != 0 && fn->stride != 1)) return POGS_EINVAL;
  const int64_t cnt = fn->stride ? len : 1;
  for (int64_t k = 0; k < cnt; ++k) {
    const double a = fn->a ? fn->a[k] : 1.0;
    const double b = fn->b ? fn->b[k] : 0.0;
    const double c = fn->c ? fn->c[k] : 1.0;
    const double d = fn->d ? fn->d[k] : 0.0;
    const double e = fn->e ? fn->e[k] : 0.0;
    if (!fn_entry_ok(fn->h[k], a, b, c, d, e)) return POGS_EINVAL;
  }
  return POGS_OK;
}

inline int expand_fn(const pogs_fn *fn, int64_t len, HostFn *out) {
  if (!fn || fn->len != len || !fn->h || (fn->stride != 0 && fn->stride != 1)) return POGS_EINVAL;
  out->h.resize(len);
  out->a.resize(len);
  out->b.resize(len);
  out->c.resize(len);
  out->d.resize(len);
  out->e.resize(len);
  for (int64_t i = 0; i < len; ++i) {
    const int64_t k = fn->stride ? i : 0;
    const uint8_t h = fn->h[k];
    const double a = fn->a ? fn->a[k] : 1.0;
    const double b = fn->b ? fn->b[k] : 0.0;
    const double c = fn->c ? fn->c[k] : 1.0;
    const double d = fn->d ? fn->d[k] : 0.0;
    const double e = fn->e ? fn->e[k] : 0.0;
    if (!fn_entry_ok(h, a, b, c, d, e)) return POGS_EINVAL;
    out->h[i] = h;
    out->a[i] = a;
    out->b[i] = b;
    out->c[i] = c;
    out->d[i] = d;
    out->e[i] = e;
  }
  return POGS_OK;
}

// Validate a pogs_fn of length len and write it expanded: h codes to h (len
// bytes) and the parameters a, b, c, d, e as five float64 arrays of len
// entries each, one after the other, at v.  Same checks as expand_fn.
inline int stage_fn(const pogs_fn *fn, int64_t len, uint8_t *h, double *v) {
  if (!fn || fn->len != len || !fn->h || (fn->stride != 0 && fn->stride != 1)) return POGS_EINVAL;
  double *va = v, *vb = v + len, *vc = v + 2 * len, *vd = v + 3 * len, *ve = v + 4 * len;
  for (int64_t i = 0; i < len; ++i) {
    const int64_t k = fn->stride ? i : 0;
    const uint8_t hk = fn->h[k];
    const double a = fn->a ? fn->a[k] : 1.0;
    const double b = fn->b ? fn->b[k] : 0.0;
    const double c = fn->c ? fn->c[k] : 1.0;
    const double d = fn->d ? fn->d[k] : 0.0;
    const double e = fn->e ? fn->e[k] : 0.0;
    if (!fn_entry_ok(hk, a, b, c, d, e)) return POGS_EINVAL;
    h[i] = hk;
    va[i] = a;
    vb[i] = b;
    vc[i] = c;
    vd[i] = d;
    ve[i] = e;
  }
  return POGS_OK;
}

inline int check_params(const pogs_params &p) {
  if (!(p.eps_abs >= 0.0) || !(p.eps_rel >= 0.0) || p.max_iter <= 0 || !(p.rho0 > 0.0) || !(p.alpha > 0.0) ||
      !(p.alpha < 2.0) || !(p.delta >= 1.0) || !(p.tau > 0.0) || !(p.tau <= 1.0) || p.equil_iters < 0 ||
      p.chunk_iters < 0 || !finite(p.eps_abs) || !finite(p.eps_rel) || !finite(p.rho0) || !finite(p.delta))
    return POGS_EINVAL;
  if (p.projection != POGS_PROJ_DIRECT && p.projection != POGS_PROJ_CGLS) return POGS_EINVAL;
  if (p.stop_rule != POGS_STOP_RESIDUAL && p.stop_rule != POGS_STOP_GAP) return POGS_EINVAL;
  if (p.sparse_segment < 0) return POGS_EINVAL;
  if (p.projection == POGS_PROJ_CGLS && (p.cg_max_iter < 1 || p.cg_max_iter > 1000 || !(p.cg_tol > 0.0) ||
                                         !finite(p.cg_tol)))
    return POGS_EINVAL;
  return POGS_OK;
}


}  // namespace pogs
