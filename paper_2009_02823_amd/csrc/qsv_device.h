// Device helpers: complex arithmetic in registers, state loads/stores, index arithmetic and the
// deterministic FP64 block reduction.
#pragma once

#include "qsv_internal.h"

namespace qsv {

template <typename R>
struct Vec2;
template <>
struct Vec2<double> {
  using T = double2;
};
template <>
struct Vec2<float> {
  using T = float2;
};

template <typename R>
struct cx {
  R r, i;
};

template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) {
  return {a.r + b.r, a.i + b.i};
}
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) {
  return {a.r - b.r, a.i - b.i};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) {
  return {s * a.r, s * a.i};
}
template <typename R>
__device__ __forceinline__ cx<R> conj(cx<R> a) {
  return {a.r, -a.i};
}
template <typename R>
__device__ __forceinline__ cx<R> neg(cx<R> a) {
  return {-a.r, -a.i};
}
// c ? a : b, selected per component (a select of whole structs would make the compiler pick
// between their addresses and keep them in scratch memory).
template <typename R>
__device__ __forceinline__ cx<R> sel(bool c, cx<R> a, cx<R> b) {
  return {c ? a.r : b.r, c ? a.i : b.i};
}

// Amplitudes live in global memory (device allocations): accessed through global-address-space
// pointers, so the compiler emits global loads and stores. Generic (flat) accesses would also
// count against the LDS counter, and waiting for them would wait for LDS reads in flight too.
#define QSV_GLOBAL __attribute__((address_space(1)))
// (clang vector types: the HIP vector structs cannot be copied through such pointers)
template <typename R>
__device__ __forceinline__ cx<R> load(const typename Vec2<R>::T* p, uint64_t j) {
  using E = R __attribute__((ext_vector_type(2)));
  const E v = ((const QSV_GLOBAL E*)p)[j];
  return {v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void store(typename Vec2<R>::T* p, uint64_t j, cx<R> a) {
  using E = R __attribute__((ext_vector_type(2)));
  E v;
  v.x = a.r;
  v.y = a.i;
  ((QSV_GLOBAL E*)p)[j] = v;
}

// Matrix entry k of a gate record, narrowed to the storage precision.
// The record (32 double2 entries) read as plain doubles through a global pointer.
__device__ __forceinline__ const QSV_GLOBAL double* rec_words(const GateRec* rec) {
  return (const QSV_GLOBAL double*)rec;
}
template <typename R>
__device__ __forceinline__ cx<R> mat(const GateRec* rec, int k) {
  const QSV_GLOBAL double* d = rec_words(rec) + 2 * k;
  return {(R)d[0], (R)d[1]};
}

// acc += conj(l) * m, evaluated in FP64 whatever the storage precision.
template <typename R>
__device__ __forceinline__ void acc_dot(double2& acc, cx<R> l, cx<R> m) {
  const double lr = l.r, li = l.i, mr = m.r, mi = m.i;
  acc.x += lr * mr + li * mi;
  acc.y += lr * mi - li * mr;
}

// Index of the g-th element of the set {j : bit q of j is 0}.
__device__ __forceinline__ uint64_t insert_zero(uint64_t g, int q) {
  const uint64_t low = g & ((1ull << q) - 1);
  return ((g >> q) << (q + 1)) | low;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Deterministic block sum of a complex FP64 value held by every thread: butterfly within each
// wave, then the waves in index order. Result written by thread 0 to *out. All threads must call.
template <int BLOCK>
__device__ __forceinline__ void block_sum_store(double2 v, double2* out) {
  __shared__ double2 sm[BLOCK / 64];
  const double re = wave_sum(v.x), im = wave_sum(v.y);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sm[w] = make_double2(re, im);
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 s = sm[0];
    for (int k = 1; k < BLOCK / 64; ++k) {
      s.x += sm[k].x;
      s.y += sm[k].y;
    }
    *out = s;
  }
  __syncthreads();
}

}  // namespace qsv
