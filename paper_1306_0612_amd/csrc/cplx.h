// Small complex helpers for device code (FP32 and FP64).
#pragma once
#include <hip/hip_runtime.h>

namespace lbs {

template <typename T>
struct cx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> mk(T a, T b) {
  return cx<T>{a, b};
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return cx<T>{a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return cx<T>{a.x - b.x, a.y - b.y};
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return cx<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) {
  return cx<T>{s * a.x, s * a.y};
}
__device__ __forceinline__ float tfma(float a, float b, float c) {
  return __builtin_fmaf(a, b, c);
}
__device__ __forceinline__ double tfma(double a, double b, double c) {
  return __builtin_fma(a, b, c);
}
// a * b + c in four fused multiply-adds, x = a.x b.x + (c.x - a.y b.y),
// y = a.x b.y + (c.y + a.y b.x): the step of a complex Horner scheme
template <typename T>
__device__ __forceinline__ cx<T> cfma(cx<T> a, cx<T> b, cx<T> c) {
  return cx<T>{tfma(a.x, b.x, tfma(-a.y, b.y, c.x)),
               tfma(a.x, b.y, tfma(a.y, b.x, c.y))};
}
template <typename T>
__device__ __forceinline__ cx<T> cinv(cx<T> a) {
  T d = T(1) / (a.x * a.x + a.y * a.y);
  return cx<T>{a.x * d, -a.y * d};
}
template <typename T>
__device__ __forceinline__ cx<T> cpow(cx<T> z, int n) {
  cx<T> r{T(1), T(0)};
  while (n) {
    if (n & 1) r = r * z;
    z = z * z;
    n >>= 1;
  }
  return r;
}

}  // namespace lbs
