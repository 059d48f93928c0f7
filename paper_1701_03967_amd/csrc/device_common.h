// Device helpers shared by the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace fftfem {

constexpr int kThreads = 256;

template <typename T>
struct C2 {
  T x, y;
};

template <typename T>
__device__ __forceinline__ C2<T> cadd(C2<T> a, C2<T> b) {
  return {a.x + b.x, a.y + b.y};
}
template <typename T>
__device__ __forceinline__ C2<T> csub(C2<T> a, C2<T> b) {
  return {a.x - b.x, a.y - b.y};
}
template <typename T>
__device__ __forceinline__ C2<T> cmul(C2<T> a, C2<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ C2<T> cmulc(C2<T> a, C2<T> b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// The hardware deals workgroups round-robin over the eight XCDs; remap so
// that consecutive tiles land on one XCD (one L2).
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  const int X = 8;
  int q = nblocks / X, r = nblocks % X;
  int xcd = bid % X, idx = bid / X;
  return (xcd < r) ? xcd * (q + 1) + idx : r * (q + 1) + (xcd - r) * q + idx;
}

template <typename T>
__device__ __forceinline__ T load_in(const void* p, int f64, int64_t i) {
  return f64 ? (T)((const double*)p)[i] : ((const T*)p)[i];
}
// kind 0: T, 1: double, 2: float
template <typename T>
__device__ __forceinline__ void store_out(void* p, int kind, int64_t i, T v) {
  if (kind == 1)
    ((double*)p)[i] = (double)v;
  else if (kind == 2)
    ((float*)p)[i] = (float)v;
  else
    ((T*)p)[i] = v;
}
// Complex FFT buffers in LDS are addressed through an XOR swizzle of the
// slot index inside aligned 256-byte blocks: slot i lives at
// i ^ ((i / B) mod B), B = 256 / sizeof(C2<T>).  Lanes that access slots B
// apart (the strided writes of the first Stockham stages) then hit
// different banks, while runs of consecutive slots stay conflict-free; the
// map is a permutation of each block, so it needs no extra space.  Every
// access to an FFT buffer goes through slot()/set_comp()/get_comp().
template <typename T>
__device__ __forceinline__ int swz(int i) {
  constexpr int LB = sizeof(T) == 8 ? 4 : 5;
  return i ^ ((i >> LB) & ((1 << LB) - 1));
}
template <typename T>
__device__ __forceinline__ C2<T>& slot(C2<T>* b, int i) {
  return b[swz<T>(i)];
}
template <typename T>
__device__ __forceinline__ const C2<T>& slot(const C2<T>* b, int i) {
  return b[swz<T>(i)];
}
template <typename T>
__device__ __forceinline__ void set_comp(C2<T>* b, int idx, int comp, T v) {
  reinterpret_cast<T*>(b + swz<T>(idx))[comp] = v;
}
template <typename T>
__device__ __forceinline__ T get_comp(const C2<T>* b, int idx, int comp) {
  return reinterpret_cast<const T*>(b + swz<T>(idx))[comp];
}

}  // namespace fftfem
