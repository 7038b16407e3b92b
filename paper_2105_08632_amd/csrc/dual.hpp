// Forward-mode dual numbers used by the HIP path.
//
//  * Dual<R>      value + one tangent: instantiating the residual kernels with
//                 it gives the exact Jacobian-vector product J(U) v.
//  * MDual<R, K>  value + K tangents: evaluates the pointwise flux Jacobians
//                 (K seeded inputs at once) for the Jacobian-block assembly.
//
// Non-smooth operations (|x|, max) branch on the value, so the derivative is
// that of the active branch; ties take the first (left) argument.
#pragma once
#include <hip/hip_runtime.h>
#include <cmath>

#define FR_HD __host__ __device__ __forceinline__

template <class R> struct Dual {
  R v, d;
  FR_HD Dual() {}
  FR_HD Dual(R a) : v(a), d(R(0)) {}
  FR_HD Dual(R a, R b) : v(a), d(b) {}
};
template <class R> FR_HD Dual<R> operator+(const Dual<R>& a, const Dual<R>& b) { return Dual<R>(a.v + b.v, a.d + b.d); }
template <class R> FR_HD Dual<R> operator-(const Dual<R>& a, const Dual<R>& b) { return Dual<R>(a.v - b.v, a.d - b.d); }
template <class R> FR_HD Dual<R> operator-(const Dual<R>& a) { return Dual<R>(-a.v, -a.d); }
template <class R> FR_HD Dual<R> operator*(const Dual<R>& a, const Dual<R>& b) { return Dual<R>(a.v * b.v, a.d * b.v + a.v * b.d); }
template <class R> FR_HD Dual<R> operator/(const Dual<R>& a, const Dual<R>& b) {
  R q = a.v / b.v;
  return Dual<R>(q, (a.d - q * b.d) / b.v);
}
template <class R> FR_HD Dual<R> operator*(R s, const Dual<R>& a) { return Dual<R>(s * a.v, s * a.d); }
template <class R> FR_HD Dual<R> operator*(const Dual<R>& a, R s) { return Dual<R>(s * a.v, s * a.d); }
template <class R> FR_HD Dual<R> operator+(const Dual<R>& a, R s) { return Dual<R>(a.v + s, a.d); }
template <class R> FR_HD Dual<R> operator-(const Dual<R>& a, R s) { return Dual<R>(a.v - s, a.d); }
template <class R> FR_HD Dual<R>& operator+=(Dual<R>& a, const Dual<R>& b) { a.v += b.v; a.d += b.d; return a; }
template <class R> FR_HD Dual<R>& operator-=(Dual<R>& a, const Dual<R>& b) { a.v -= b.v; a.d -= b.d; return a; }

template <class R, int K> struct MDual {
  R v, d[K];
  FR_HD MDual() {}
  FR_HD MDual(R a) : v(a) {
#pragma unroll
    for (int k = 0; k < K; ++k) d[k] = R(0);
  }
};
template <class R, int K> FR_HD MDual<R, K> operator+(const MDual<R, K>& a, const MDual<R, K>& b) {
  MDual<R, K> r; r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <class R, int K> FR_HD MDual<R, K> operator-(const MDual<R, K>& a, const MDual<R, K>& b) {
  MDual<R, K> r; r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <class R, int K> FR_HD MDual<R, K> operator-(const MDual<R, K>& a) {
  MDual<R, K> r; r.v = -a.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
  return r;
}
template <class R, int K> FR_HD MDual<R, K> operator*(const MDual<R, K>& a, const MDual<R, K>& b) {
  MDual<R, K> r; r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <class R, int K> FR_HD MDual<R, K> operator/(const MDual<R, K>& a, const MDual<R, K>& b) {
  MDual<R, K> r; r.v = a.v / b.v;
  R ib = R(1) / b.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
  return r;
}
template <class R, int K> FR_HD MDual<R, K> operator*(R s, const MDual<R, K>& a) {
  MDual<R, K> r; r.v = s * a.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = s * a.d[k];
  return r;
}
template <class R, int K> FR_HD MDual<R, K> operator*(const MDual<R, K>& a, R s) { return s * a; }
template <class R, int K> FR_HD MDual<R, K> operator+(const MDual<R, K>& a, R s) { MDual<R, K> r = a; r.v += s; return r; }
template <class R, int K> FR_HD MDual<R, K> operator-(const MDual<R, K>& a, R s) { MDual<R, K> r = a; r.v -= s; return r; }
template <class R, int K> FR_HD MDual<R, K>& operator+=(MDual<R, K>& a, const MDual<R, K>& b) { a = a + b; return a; }
template <class R, int K> FR_HD MDual<R, K>& operator-=(MDual<R, K>& a, const MDual<R, K>& b) { a = a - b; return a; }

// ---- uniform helpers over float / double / Dual / MDual
FR_HD float val(float x) { return x; }
FR_HD double val(double x) { return x; }
template <class R> FR_HD R val(const Dual<R>& x) { return x.v; }
template <class R, int K> FR_HD R val(const MDual<R, K>& x) { return x.v; }

FR_HD float fr_sqrt(float x) { return sqrtf(x); }
FR_HD double fr_sqrt(double x) { return sqrt(x); }
template <class R> FR_HD Dual<R> fr_sqrt(const Dual<R>& x) {
  R s = fr_sqrt(x.v);
  return Dual<R>(s, x.d / (R(2) * s));
}
template <class R, int K> FR_HD MDual<R, K> fr_sqrt(const MDual<R, K>& x) {
  MDual<R, K> r; r.v = fr_sqrt(x.v);
  R h = R(0.5) / r.v;
#pragma unroll
  for (int k = 0; k < K; ++k) r.d[k] = x.d[k] * h;
  return r;
}
template <class T> FR_HD T fr_abs(const T& x) { return val(x) >= 0 ? x : -x; }
template <class T> FR_HD T fr_max(const T& a, const T& b) { return val(a) >= val(b) ? a : b; }

// Base real type of a scalar.
template <class T> struct BaseOf { typedef T type; };
template <class R> struct BaseOf<Dual<R>> { typedef R type; };
template <class R, int K> struct BaseOf<MDual<R, K>> { typedef R type; };
