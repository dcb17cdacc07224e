// Forward-mode dual numbers for the adjoint kernels: value plus N partial
// derivatives, FP64.  Pair functions are written once, templated on the
// scalar type, and differentiated by seeding the inputs.
#pragma once

#include <hip/hip_runtime.h>

namespace pbmp {

template <int N> struct Dual {
  double v;
  double d[N];
  __host__ __device__ Dual() : v(0.0) {
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
  __host__ __device__ Dual(double x) : v(x) {
    for (int i = 0; i < N; ++i) d[i] = 0.0;
  }
  __host__ __device__ static Dual var(double x, int k) {
    Dual r(x);
    r.d[k] = 1.0;
    return r;
  }
};

template <int N> __device__ inline Dual<N> operator+(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a.v + b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i];
  return r;
}
template <int N> __device__ inline Dual<N> operator-(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a.v - b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i];
  return r;
}
template <int N> __device__ inline Dual<N> operator-(const Dual<N> &a) {
  Dual<N> r;
  r.v = -a.v;
  for (int i = 0; i < N; ++i) r.d[i] = -a.d[i];
  return r;
}
template <int N> __device__ inline Dual<N> operator*(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a.v * b.v;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i];
  return r;
}
template <int N> __device__ inline Dual<N> operator/(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  const double ib = 1.0 / b.v;
  r.v = a.v * ib;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib;
  return r;
}
template <int N> __device__ inline Dual<N> operator+(const Dual<N> &a, double b) {
  Dual<N> r = a;
  r.v += b;
  return r;
}
template <int N> __device__ inline Dual<N> operator+(double b, const Dual<N> &a) { return a + b; }
template <int N> __device__ inline Dual<N> operator-(const Dual<N> &a, double b) {
  Dual<N> r = a;
  r.v -= b;
  return r;
}
template <int N> __device__ inline Dual<N> operator-(double b, const Dual<N> &a) {
  Dual<N> r = -a;
  r.v += b;
  return r;
}
template <int N> __device__ inline Dual<N> operator*(const Dual<N> &a, double b) {
  Dual<N> r;
  r.v = a.v * b;
  for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b;
  return r;
}
template <int N> __device__ inline Dual<N> operator*(double b, const Dual<N> &a) { return a * b; }
template <int N> __device__ inline Dual<N> operator/(const Dual<N> &a, double b) {
  return a * (1.0 / b);
}
template <int N> __device__ inline Dual<N> operator/(double a, const Dual<N> &b) {
  return Dual<N>(a) / b;
}
template <int N> __device__ inline Dual<N> &operator+=(Dual<N> &a, const Dual<N> &b) {
  a = a + b;
  return a;
}
template <int N> __device__ inline Dual<N> &operator-=(Dual<N> &a, const Dual<N> &b) {
  a = a - b;
  return a;
}

template <int N> __device__ inline Dual<N> chain(const Dual<N> &a, double f, double df) {
  Dual<N> r;
  r.v = f;
  for (int i = 0; i < N; ++i) r.d[i] = df * a.d[i];
  return r;
}
template <int N> __device__ inline Dual<N> sqrt(const Dual<N> &a) {
  const double s = ::sqrt(a.v);
  return chain(a, s, 0.5 / s);
}
template <int N> __device__ inline Dual<N> exp(const Dual<N> &a) {
  const double e = ::exp(a.v);
  return chain(a, e, e);
}
template <int N> __device__ inline Dual<N> expm1(const Dual<N> &a) {
  return chain(a, ::expm1(a.v), ::exp(a.v));
}
template <int N> __device__ inline Dual<N> asinh(const Dual<N> &a) {
  return chain(a, ::asinh(a.v), 1.0 / ::sqrt(1.0 + a.v * a.v));
}
template <int N> __device__ inline Dual<N> cosh(const Dual<N> &a) {
  return chain(a, ::cosh(a.v), ::sinh(a.v));
}

// keep the plain-double math functions visible next to the dual overloads
using ::asinh;
using ::cosh;
using ::exp;
using ::expm1;
using ::sqrt;

__device__ inline double value_of(double x) { return x; }
template <int N> __device__ inline double value_of(const Dual<N> &x) { return x.v; }

}  // namespace pbmp
