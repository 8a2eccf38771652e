// Forward-mode dual numbers with K directional derivatives (device and host).
// Used for the local Jacobians of the Riemann solvers in the adjoint kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace dgfv {

template <int K>
struct Dual {
  double v;
  double d[K];

  __host__ __device__ Dual() : v(0.0) {
    for (int k = 0; k < K; ++k) d[k] = 0.0;
  }
  __host__ __device__ Dual(double x) : v(x) {  // NOLINT: implicit constants
    for (int k = 0; k < K; ++k) d[k] = 0.0;
  }
  __host__ __device__ static Dual seed(double x, int k) {
    Dual r(x);
    r.d[k] = 1.0;
    return r;
  }
};

template <int K>
__host__ __device__ inline Dual<K> operator+(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r;
  r.v = a.v + b.v;
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int K>
__host__ __device__ inline Dual<K> operator-(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r;
  r.v = a.v - b.v;
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int K>
__host__ __device__ inline Dual<K> operator-(const Dual<K>& a) {
  Dual<K> r;
  r.v = -a.v;
  for (int k = 0; k < K; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int K>
__host__ __device__ inline Dual<K> operator*(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r;
  r.v = a.v * b.v;
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int K>
__host__ __device__ inline Dual<K> operator/(const Dual<K>& a, const Dual<K>& b) {
  Dual<K> r;
  const double ib = 1.0 / b.v;
  r.v = a.v * ib;
  for (int k = 0; k < K; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
  return r;
}
template <int K> __host__ __device__ inline Dual<K> operator+(const Dual<K>& a, double b) { return a + Dual<K>(b); }
template <int K> __host__ __device__ inline Dual<K> operator+(double a, const Dual<K>& b) { return Dual<K>(a) + b; }
template <int K> __host__ __device__ inline Dual<K> operator-(const Dual<K>& a, double b) { return a - Dual<K>(b); }
template <int K> __host__ __device__ inline Dual<K> operator-(double a, const Dual<K>& b) { return Dual<K>(a) - b; }
template <int K>
__host__ __device__ inline Dual<K> operator*(const Dual<K>& a, double b) {
  Dual<K> r;
  r.v = a.v * b;
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * b;
  return r;
}
template <int K> __host__ __device__ inline Dual<K> operator*(double a, const Dual<K>& b) { return b * a; }
template <int K> __host__ __device__ inline Dual<K> operator/(const Dual<K>& a, double b) { return a * (1.0 / b); }
template <int K> __host__ __device__ inline Dual<K> operator/(double a, const Dual<K>& b) { return Dual<K>(a) / b; }

template <int K>
__host__ __device__ inline Dual<K> sqrt(const Dual<K>& a) {
  Dual<K> r;
  r.v = ::sqrt(a.v);
  const double h = 0.5 / r.v;
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * h;
  return r;
}
template <int K>
__host__ __device__ inline Dual<K> log(const Dual<K>& a) {
  Dual<K> r;
  r.v = ::log(a.v);
  const double ia = 1.0 / a.v;
  for (int k = 0; k < K; ++k) r.d[k] = a.d[k] * ia;
  return r;
}
// Derivative of the branch taken (ties take the first argument).
template <int K>
__host__ __device__ inline Dual<K> fabs(const Dual<K>& a) { return a.v < 0.0 ? -a : a; }
template <int K>
__host__ __device__ inline Dual<K> fmax(const Dual<K>& a, const Dual<K>& b) { return b.v > a.v ? b : a; }
template <int K> __host__ __device__ inline Dual<K> fmax(double a, const Dual<K>& b) { return fmax(Dual<K>(a), b); }
template <int K> __host__ __device__ inline Dual<K> fmax(const Dual<K>& a, double b) { return fmax(a, Dual<K>(b)); }

template <int K> __host__ __device__ inline bool operator<(const Dual<K>& a, const Dual<K>& b) { return a.v < b.v; }
template <int K> __host__ __device__ inline bool operator<(const Dual<K>& a, double b) { return a.v < b; }
template <int K> __host__ __device__ inline bool operator>(const Dual<K>& a, double b) { return a.v > b; }

__host__ __device__ inline double value(double x) { return x; }
template <int K> __host__ __device__ inline double value(const Dual<K>& x) { return x.v; }

}  // namespace dgfv
