// Device helpers shared by the gfx950 kernel sources of the Spectral Ewald
// k-space path.
#pragma once
#include <hip/hip_runtime.h>

#include "se_internal.h"

namespace se {

template <typename T>
struct __align__(2 * sizeof(T)) cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) {
  return {a.re + b.re, a.im + b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) {
  return {a.re - b.re, a.im - b.im};
}
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cscale(cx<T> a, T s) {
  return {a.re * s, a.im * s};
}
// multiply by sign * i
template <typename T>
__device__ __forceinline__ cx<T> mul_si(cx<T> a, int sign) {
  return sign > 0 ? cx<T>{-a.im, a.re} : cx<T>{a.im, -a.re};
}

template <typename T>
struct Quad {
  T fx, fy, fz, q;
};

// Pointers held in descriptors are generic (they could address LDS), so
// loads through them are flat vector loads.  Device buffers are global
// memory: these casts let the compiler use global (and, for uniform
// addresses, scalar) loads and stores.
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gld(const T* p) {
  return (const __attribute__((address_space(1))) T*)(p);
}
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gst(T* p) {
  return (__attribute__((address_space(1))) T*)(p);
}

// Complex values through global pointers, as two-component vectors.
template <typename T>
using vec2 = T __attribute__((ext_vector_type(2)));
template <typename T>
__device__ __forceinline__ cx<T> ld_cx(const cx<T>* p, long long i) {
  const vec2<T> v = gld(reinterpret_cast<const vec2<T>*>(p))[i];
  return cx<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void st_cx(cx<T>* p, long long i, cx<T> v) {
  gst(reinterpret_cast<vec2<T>*>(p))[i] = vec2<T>{v.re, v.im};
}
template <typename T>
using vec4 = T __attribute__((ext_vector_type(4)));
template <typename T>
__device__ __forceinline__ Quad<T> ld_quad(const void* p, long long i) {
  const vec4<T> v = gld(reinterpret_cast<const vec4<T>*>(p))[i];
  return Quad<T>{v.x, v.y, v.z, v.w};
}

// Quotient of small non-negative integers a < 2^21 by d, given inv_d = 1/d in
// FP32: (a + 1/2)/d lies at least 1/(2d) from an integer, which exceeds the
// rounding error of the product, so truncation gives floor(a/d) exactly.
__device__ __forceinline__ int fdiv(int a, float inv_d) { return (int)(((float)a + 0.5f) * inv_d); }

// Work item of workgroup b out of n.  Workgroups are handed to the 8 XCDs in
// turn (b mod 8), so neighbouring items, which share cache lines at their
// edges, land in different L2s.  Mode 1 gives each XCD one contiguous range of
// items; mode c >= 2 gives each XCD chunks of c neighbouring items while the
// XCDs work side by side (rounds of 8c items; the last partial round keeps the
// plain order).  Both are bijections of [0, n); mode 0 is the plain order.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_item(int b, int n, int mode) {
  const int x = b % kXcds, s = b / kXcds;
  if (mode == 1) {
    const int q = n / kXcds, r = n % kXcds;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + s;
  }
  const int c = mode, round = kXcds * c;
  if (b >= (n / round) * round) return b;
  return ((s / c) * kXcds + x) * c + s % c;
}
__device__ __forceinline__ int work_item(int mode) {
  return mode > 0 ? xcd_item(blockIdx.x, gridDim.x, mode) : blockIdx.x;
}

}  // namespace se
