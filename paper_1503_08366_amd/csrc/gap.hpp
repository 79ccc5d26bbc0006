// Values and conjugates of the parametric functions of Section 5 for the
// gap-based stopping rule of Section 3.4: eta = f(y) + g(x) + f*(nu) + g*(mu)
// on a primal and dual feasible tuple.  Every indicator is exact here (+inf
// outside its set), so the gap is infinite whenever a constraint is violated.
#pragma once

#include "prox.hpp"

namespace pogs {

// h(u), +inf outside the domain of h.
__device__ inline double h_value_strict(int h, double u) {
  const double inf = __builtin_huge_val();
  switch (h) {
    case kZero: return 0.0;
    case kIdentity: return u;
    case kAbs: return fabs(u);
    case kSquare: return 0.5 * u * u;
    case kHuber: return fabs(u) <= 1.0 ? 0.5 * u * u : fabs(u) - 0.5;
    case kHinge: return u > 0.0 ? u : 0.0;
    case kLogistic: return u > 0.0 ? u + log1p(exp(-u)) : log1p(exp(u));
    case kIndGe0: return u >= 0.0 ? 0.0 : inf;
    case kIndLe0: return u <= 0.0 ? 0.0 : inf;
    case kIndEq0: return u == 0.0 ? 0.0 : inf;
    case kIndBox01: return (u >= 0.0 && u <= 1.0) ? 0.0 : inf;
    case kExp: return exp(u);
    case kNegEntr: return u > 0.0 ? u * log(u) : (u == 0.0 ? 0.0 : inf);
    case kNegLog: return u > 0.0 ? -log(u) : inf;
    case kRecipr: return u > 0.0 ? 1.0 / u : inf;
    case kMaxNeg0: return u < 0.0 ? -u : 0.0;
    default: return inf;
  }
}

// h*(s) = sup_u s u - h(u) (textbook conjugates), +inf outside their domains.
__device__ inline double h_conj(int h, double s) {
  const double inf = __builtin_huge_val();
  switch (h) {
    case kZero: return s == 0.0 ? 0.0 : inf;
    case kIdentity: return s == 1.0 ? 0.0 : inf;
    case kAbs: return fabs(s) <= 1.0 ? 0.0 : inf;
    case kSquare: return 0.5 * s * s;
    case kHuber: return fabs(s) <= 1.0 ? 0.5 * s * s : inf;
    case kHinge: return (s >= 0.0 && s <= 1.0) ? 0.0 : inf;
    case kLogistic:
      if (s < 0.0 || s > 1.0) return inf;
      return (s > 0.0 ? s * log(s) : 0.0) + (s < 1.0 ? (1.0 - s) * log1p(-s) : 0.0);
    case kIndGe0: return s <= 0.0 ? 0.0 : inf;
    case kIndLe0: return s >= 0.0 ? 0.0 : inf;
    case kIndEq0: return 0.0;
    case kIndBox01: return s > 0.0 ? s : 0.0;
    case kExp: return s > 0.0 ? s * log(s) - s : (s == 0.0 ? 0.0 : inf);
    case kNegEntr: return exp(s - 1.0);
    case kNegLog: return s < 0.0 ? -1.0 - log(-s) : inf;
    case kRecipr: return s <= 0.0 ? -2.0 * sqrt(-s) : inf;
    case kMaxNeg0: return (s >= -1.0 && s <= 0.0) ? 0.0 : inf;
    default: return inf;
  }
}

// f(y) = c h(a y - b) + d y + (e/2) y^2 with exact indicators (c = 0: no h term).
__device__ inline double fn_value_strict(int h, double a, double b, double c, double d, double e, double y) {
  const double hv = c > 0.0 ? c * h_value_strict(h, a * y - b) : 0.0;
  return hv + d * y + 0.5 * e * y * y;
}

// f*(nu) = sup_y nu y - f(y).  With s = nu - d:
//   e = 0: c h*(s / (a c)) + b s / a  (c > 0), the indicator of {s = 0} (c = 0);
//   e > 0: s^2 / (2e) (c = 0), else s y* - (e/2) y*^2 - c h(a y* - b) with
//          y* = argmin_y c h(a y - b) + (e/2)(y - s/e)^2 (the prox of the h term
//          with penalty e at s/e), where the supremum is attained.
__device__ inline double fn_conj_value(int h, double a, double b, double c, double d, double e, double nu) {
  const double s = nu - d;
  if (e == 0.0) {
    if (c == 0.0) return s == 0.0 ? 0.0 : __builtin_huge_val();
    return c * h_conj(h, s / (a * c)) + b * s / a;
  }
  if (c == 0.0) return s * s / (2.0 * e);
  const double y = prox_param<double>(h, a, b, c, 0.0, 0.0, s / e, e);
  return s * y - 0.5 * e * y * y - c * h_value_strict(h, a * y - b);
}

}  // namespace pogs
