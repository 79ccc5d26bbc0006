// Proximal operators of the parametric separable functions of Section 5,
//   f(y) = c h(a y - b) + d y + (e/2) y^2,
// evaluated elementwise on the device.
#pragma once

#include "common.hpp"

namespace pogs {

enum HCode : int {
  kZero = 0, kIdentity = 1, kAbs = 2, kSquare = 3, kHuber = 4, kHinge = 5,
  kLogistic = 6, kIndGe0 = 7, kIndLe0 = 8, kIndEq0 = 9, kIndBox01 = 10,
  kExp = 11, kNegEntr = 12, kNegLog = 13, kRecipr = 14, kMaxNeg0 = 15,
  kNumH = 16
};

__device__ inline float fexp(float x) { return __expf(x); }
__device__ inline double fexp(double x) { return exp(x); }

// Root of sigma(u) + r (u - z) = 0, i.e. argmin_u log(1 + e^u) + (r/2)(u - z)^2.
// The left side increases in u and changes sign on [z - 1/r, z].  Safeguarded
// Newton: each evaluation shrinks the bracket; a Newton step is taken only if
// it stays inside the bracket and is less than half the previous step,
// otherwise the bracket is bisected.  So the bracket at least halves every
// two iterations and the loop cannot cycle.  Fixed cap on the iteration count.
template <typename T> __device__ inline T prox_logistic(T z, T r) {
  T lo = z - T(1) / r, hi = z;
  // first guess: one fixed-point step from z
  T u = z - (T(1) / (T(1) + fexp(-z))) / r;
  if (!(u > lo && u < hi)) u = T(0.5) * (lo + hi);
  const T tol = sizeof(T) == 4 ? T(1e-7) : T(1e-15);
  T last = hi - lo;  // length of the previous step
  for (int it = 0; it < 100; ++it) {
    const T s = T(1) / (T(1) + fexp(-u));
    const T g = s + r * (u - z);
    if (g == T(0)) break;
    if (g > T(0)) hi = u; else lo = u;
    const T newton = g / (s * (T(1) - s) + r);
    T un = u - newton;
    if (!(un > lo && un < hi) || T(2) * fabs(newton) > last) un = T(0.5) * (lo + hi);
    last = fabs(un - u);
    u = un;
    const T scale = fmax(T(1), fabs(u));
    if (last <= tol * scale || hi - lo <= tol * scale) break;
  }
  return u;
}

// Root of an increasing function g on [lo, hi] (g(lo) < 0 < g(hi)) from the
// start u in the bracket, by the same safeguarded Newton iteration:
// g(u, &value, &derivative).
template <typename T, class G> __device__ inline T safe_newton(G g, T lo, T hi, T u) {
  const T tol = sizeof(T) == 4 ? T(1e-7) : T(1e-15);
  if (!(u > lo && u < hi)) u = T(0.5) * (lo + hi);
  T last = hi - lo;
  for (int it = 0; it < 100; ++it) {
    T v, dv;
    g(u, v, dv);
    if (v == T(0)) break;
    if (v > T(0)) hi = u; else lo = u;
    const T newton = v / dv;
    T un = u - newton;
    if (!(un > lo && un < hi) || T(2) * fabs(newton) > last) un = T(0.5) * (lo + hi);
    last = fabs(un - u);
    u = un;
    const T scale = fmax(T(1), fabs(u));
    if (last <= tol * scale || hi - lo <= tol * scale) break;
  }
  return u;
}

// argmin e^u + (r/2)(u - z)^2: e^u + r (u - z) increases in u, is positive
// at z and negative at z - e^z / r.
template <typename T> __device__ inline T prox_exp(T z, T r) {
  const T ez = fexp(fmin(z, T(sizeof(T) == 4 ? 80 : 700)));
  const T lo = z - ez / r, hi = z;
  return safe_newton<T>([&](T u, T &v, T &dv) {
    const T eu = fexp(u);
    v = eu + r * (u - z);
    dv = eu + r;
  }, lo, hi, z - ez / (ez + r));
}

// argmin u log u + (r/2)(u - z)^2 over u >= 0: with u = e^t the condition is
// t + r e^t - (r z - 1) = 0, increasing in t; non-negative at
// t_hi = min(r z - 1, log max(z, 1/e)) and negative at r z - 1 - r e^t_hi.
template <typename T> __device__ inline T prox_neg_entr(T z, T r) {
  const T c = r * z - T(1);
  const T thi = fmin(c, log(fmax(z, T(0.36787944117144233))));
  const T tlo = c - r * fexp(thi);
  const T t = safe_newton<T>([&](T t, T &v, T &dv) {
    const T et = fexp(t);
    v = t + r * et - c;
    dv = T(1) + r * et;
  }, tlo, thi, thi);
  return fexp(t);
}

// argmin -log u + (r/2)(u - z)^2: the positive root of r u^2 - r z u - 1,
// written without cancellation for z < 0.
template <typename T> __device__ inline T prox_neg_log(T z, T r) {
  const T s = sqrt(z * z + T(4) / r);
  return z >= T(0) ? T(0.5) * (z + s) : T(2) / (r * (s - z));
}

// argmin 1/u + (r/2)(u - z)^2 over u > 0: r (u - z) - 1/u^2 increases in u,
// is non-negative at hi = max(z, 0) + r^(-1/3) and negative at
// 1 / sqrt(r (hi - z)).
template <typename T> __device__ inline T prox_recipr(T z, T r) {
  const T hi = fmax(z, T(0)) + T(1) / cbrt(r);
  const T lo = fmin(T(1) / sqrt(r * (hi - z)), hi);
  return safe_newton<T>([&](T u, T &v, T &dv) {
    const T iu = T(1) / u;
    v = r * (u - z) - iu * iu;
    dv = r + T(2) * iu * iu * iu;
  }, lo, hi, hi);
}

// prox_{h,r}(z) = argmin_u h(u) + (r/2)(u - z)^2.
template <typename T> __device__ inline T prox_h(int h, T z, T r) {
  switch (h) {
    case kZero: return z;
    case kIdentity: return z - T(1) / r;
    case kAbs: {
      const T t = T(1) / r;
      return z > t ? z - t : (z < -t ? z + t : T(0));
    }
    case kSquare: return r * z / (T(1) + r);
    case kHuber: {
      const T t = T(1) / r;
      if (fabs(z) <= T(1) + t) return r * z / (T(1) + r);
      return z > T(0) ? z - t : z + t;
    }
    case kHinge: {
      const T t = T(1) / r;
      return z > t ? z - t : (z < T(0) ? z : T(0));
    }
    case kLogistic: return prox_logistic(z, r);
    case kIndGe0: return z > T(0) ? z : T(0);
    case kIndLe0: return z < T(0) ? z : T(0);
    case kIndEq0: return T(0);
    case kIndBox01: return z < T(0) ? T(0) : (z > T(1) ? T(1) : z);
    case kExp: return prox_exp(z, r);
    case kNegEntr: return prox_neg_entr(z, r);
    case kNegLog: return prox_neg_log(z, r);
    case kRecipr: return prox_recipr(z, r);
    case kMaxNeg0: {
      const T t = T(1) / r;
      return z < -t ? z + t : (z > T(0) ? z : T(0));
    }
    default: return z;
  }
}

// prox of c h(a y - b) + d y + (e/2) y^2 with penalty rho (Section 5):
//   (1/a) (prox_{h, (e+rho)/(c a^2)}(a (rho v - d)/(e + rho) - b) + b);
// with c == 0 the h term is absent and the result is (rho v - d)/(e + rho).
template <typename T>
__device__ inline T prox_param(int h, T a, T b, T c, T d, T e, T v, T rho) {
  const T vq = (rho * v - d) / (e + rho);
  if (!(c > T(0))) return vq;
  const T r = (e + rho) / (c * a * a);
  return (prox_h(h, a * vq - b, r) + b) / a;
}

// Value of the finite part of c h(a y - b) + d y + (e/2) y^2; indicator terms
// and the domain constraints of u log u, -log u and 1/u contribute 0 (prox
// outputs satisfy them up to rounding).
__device__ inline double fn_value(int h, double a, double b, double c, double d, double e, double y) {
  const double u = a * y - b;
  double hv = 0.0;
  switch (h) {
    case kIdentity: hv = u; break;
    case kAbs: hv = fabs(u); break;
    case kSquare: hv = 0.5 * u * u; break;
    case kHuber: hv = fabs(u) <= 1.0 ? 0.5 * u * u : fabs(u) - 0.5; break;
    case kHinge: hv = u > 0.0 ? u : 0.0; break;
    case kLogistic: hv = u > 0.0 ? u + log1p(exp(-u)) : log1p(exp(u)); break;
    case kExp: hv = exp(u); break;
    case kNegEntr: hv = u > 0.0 ? u * log(u) : 0.0; break;
    case kNegLog: hv = u > 0.0 ? -log(u) : 0.0; break;
    case kRecipr: hv = u > 0.0 ? 1.0 / u : 0.0; break;
    case kMaxNeg0: hv = u < 0.0 ? -u : 0.0; break;
    default: hv = 0.0; break;
  }
  return (c > 0.0 ? c * hv : 0.0) + d * y + 0.5 * e * y * y;
}

}  // namespace pogs
