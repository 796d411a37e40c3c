// Accumulators of the assembly kernels (resident and chunked): float64 sums,
// or float32 Kahan sums whose exact value s - c is read in float64, and the
// scaled distance r = sqrt(s) / rho in the precision of phi.
#pragma once

#include "common.h"

namespace rbf {

template <typename T>
struct Acc;
template <>
struct Acc<double> {
  double s = 0.0;
  __device__ __forceinline__ void add(double v) { s += v; }
  __device__ __forceinline__ double value() const { return s; }
};
template <>
struct Acc<float> {
  Kahan32 k;
  __device__ __forceinline__ void add(float v) { k.add(v); }
  __device__ __forceinline__ float value() const { return k.s; }
};

template <typename T>
__device__ __forceinline__ T scaled_r(double s, double irho);
template <>
__device__ __forceinline__ double scaled_r<double>(double s, double irho) {
  return __builtin_sqrt(s) * irho;
}
template <>
__device__ __forceinline__ float scaled_r<float>(double s, double irho) {
  return __builtin_sqrtf((float)s) * (float)irho;
}

// Plain-data copy of an accumulator (LDS variables take no initialisers).
template <typename T>
struct AccPod {
  T s, c;
};
__device__ __forceinline__ Acc<double> from_pod(const AccPod<double>& p) {
  Acc<double> a;
  a.s = p.s;
  return a;
}
__device__ __forceinline__ Acc<float> from_pod(const AccPod<float>& p) {
  Acc<float> a;
  a.k.s = p.s;
  a.k.c = p.c;
  return a;
}
__device__ __forceinline__ AccPod<double> to_pod(const Acc<double>& a) { return {a.s, 0.0}; }
__device__ __forceinline__ AccPod<float> to_pod(const Acc<float>& a) { return {a.k.s, a.k.c}; }

template <typename T>
__device__ __forceinline__ double partial_value(const Acc<T>& a);
template <>
__device__ __forceinline__ double partial_value<double>(const Acc<double>& a) {
  return a.s;
}
template <>
__device__ __forceinline__ double partial_value<float>(const Acc<float>& a) {
  return (double)a.k.s - (double)a.k.c;
}

}  // namespace rbf
