// Forward-mode derivatives in FP64: a value with N tangents.  The touching-
// pair block is a fixed sequence of arithmetic, square roots, logarithms,
// arctangents and sines; carried through it, Dual<N> gives the exact
// derivatives (to rounding) of that sequence along N seeded directions at
// once.  The d_* functions take double or Dual<N>, so one template body
// serves the plain FP64 evaluation and its derivatives.
#pragma once

#include <hip/hip_runtime.h>

namespace mf {

template <int N>
struct Dual {
  double v;
  double d[N];
  __device__ Dual() {}
  __device__ Dual(double x) : v(x) {
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = 0.0;
  }
};

__device__ __forceinline__ double val(double x) { return x; }
template <int N>
__device__ __forceinline__ double val(const Dual<N> &x) { return x.v; }

template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N> &a) {
  Dual<N> r;
  r.v = -a.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator+(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator+(const Dual<N> &a, double b) {
  Dual<N> r = a;
  r.v = a.v + b;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator+(double a, const Dual<N> &b) {
  return b + a;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N> &a, double b) {
  Dual<N> r = a;
  r.v = a.v - b;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(double a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a - b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = -b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(const Dual<N> &a, double b) {
  Dual<N> r;
  r.v = a.v * b;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(double a, const Dual<N> &b) {
  return b * a;
}
template <int N>
__device__ __forceinline__ Dual<N> operator/(const Dual<N> &a, const Dual<N> &b) {
  Dual<N> r;
  const double ib = 1.0 / b.v;
  r.v = a.v / b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator/(const Dual<N> &a, double b) {
  Dual<N> r;
  const double ib = 1.0 / b;
  r.v = a.v / b;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * ib;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator/(double a, const Dual<N> &b) {
  return Dual<N>(a) / b;
}
template <int N, class U>
__device__ __forceinline__ Dual<N> &operator+=(Dual<N> &a, const U &b) {
  return a = a + b;
}
template <int N, class U>
__device__ __forceinline__ Dual<N> &operator-=(Dual<N> &a, const U &b) {
  return a = a - b;
}
template <int N, class U>
__device__ __forceinline__ Dual<N> &operator*=(Dual<N> &a, const U &b) {
  return a = a * b;
}
template <int N, class U>
__device__ __forceinline__ Dual<N> &operator/=(Dual<N> &a, const U &b) {
  return a = a / b;
}

// Elementary functions.  d_sqrt of an exact zero has zero tangents: the
// callers take it only of a distance that vanishes identically (a point and
// itself), whose derivative is zero.  d_fabs of an exact zero likewise.
__device__ __forceinline__ double d_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ double d_log(double x) { return log(x); }
__device__ __forceinline__ double d_atan(double x) { return atan(x); }
__device__ __forceinline__ double d_fabs(double x) { return fabs(x); }
__device__ __forceinline__ void d_sincos(double x, double *s, double *c) { sincos(x, s, c); }

template <int N>
__device__ __forceinline__ Dual<N> d_sqrt(const Dual<N> &x) {
  Dual<N> r;
  r.v = sqrt(x.v);
  const double f = r.v > 0.0 ? 0.5 / r.v : 0.0;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = x.d[k] * f;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> d_log(const Dual<N> &x) {
  Dual<N> r;
  r.v = log(x.v);
  const double f = 1.0 / x.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = x.d[k] * f;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> d_atan(const Dual<N> &x) {
  Dual<N> r;
  r.v = atan(x.v);
  const double f = 1.0 / (1.0 + x.v * x.v);
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = x.d[k] * f;
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> d_fabs(const Dual<N> &x) {
  if (x.v > 0.0) return x;
  if (x.v < 0.0) return -x;
  return Dual<N>(0.0);
}
template <int N>
__device__ __forceinline__ void d_sincos(const Dual<N> &x, Dual<N> *s, Dual<N> *c) {
  double sv, cv;
  sincos(x.v, &sv, &cv);
  s->v = sv;
  c->v = cv;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    s->d[k] = x.d[k] * cv;
    c->d[k] = -x.d[k] * sv;
  }
}

}  // namespace mf
