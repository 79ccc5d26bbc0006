// Proximal operators of the parametric separable functions of Section 5,
//   f(y) = c h(a y - b) + d y + (e/2) y^2,
// evaluated elementwise on the device.
#pragma once

#include "common.hpp"

namespace pogs {

enum HCode : int {
  kZero = 0, kIdentity = 1, kAbs = 2, kSquare = 3, kHuber = 4, kHinge = 5,
  kLogistic = 6, kIndGe0 = 7, kIndLe0 = 8, kIndEq0 = 9, kIndBox01 = 10,
  kNumH = 11
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
// contribute 0 (prox outputs satisfy them up to rounding).
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
    default: hv = 0.0; break;
  }
  return (c > 0.0 ? c * hv : 0.0) + d * y + 0.5 * e * y * y;
}

}  // namespace pogs
