// Device helpers shared by the 2D sweep kernels: weight containers, the
// FMA, the tap masks, 16-byte vector loads and stores, periodic wrap and the
// XCD-aware block numbering.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace stencil {
namespace k2d {

// Weights passed by value in the kernel arguments (read through the
// scalar cache), or from a uniform global pointer (batched tiles).
template <typename T, int N>
struct WArr {
  T v[N];
  __device__ __forceinline__ T operator[](int i) const { return v[i]; }
};

template <typename T>
struct WPtr {
  const T *__restrict__ p;
  __device__ __forceinline__ T operator[](int i) const { return p[i]; }
};

__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <int MASK, int R>
__host__ __device__ constexpr bool in_mask(int oy, int ox) {
  return MASK == MASK_BOX ? true
         : MASK == MASK_DIAMOND ? ((oy < 0 ? -oy : oy) + (ox < 0 ? -ox : ox) <= R)
                                : (oy == 0 || ox == 0);
}

template <typename T, int VX>
struct Vec {
  T v[VX];
};

// Streaming accesses: every grid value is loaded once per sweep (halo rows
// and columns aside) and every output stored once, so both use nontemporal
// hints; on gfx950 this raises streaming bandwidth by about a tenth.
template <typename T, int VX>
__device__ __forceinline__ void load_vec(const T *__restrict__ p, T (&d)[VX]) {
  if constexpr (VX * sizeof(T) % 16 == 0) {
    constexpr int E = 16 / sizeof(T);  // elements per 16-byte chunk
    using V = __attribute__((ext_vector_type(E))) T;
#pragma unroll
    for (int c = 0; c < VX / E; ++c) {
      V t = __builtin_nontemporal_load(reinterpret_cast<const V *>(p + c * E));
#pragma unroll
      for (int i = 0; i < E; ++i) d[c * E + i] = t[i];
    }
  } else if constexpr (VX * sizeof(T) == 8) {
    using V = __attribute__((ext_vector_type(8 / sizeof(T)))) T;
    V t = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
#pragma unroll
    for (int i = 0; i < VX; ++i) d[i] = t[i];
  } else {
#pragma unroll
    for (int i = 0; i < VX; ++i) d[i] = __builtin_nontemporal_load(p + i);
  }
}

template <typename T, int VX>
__device__ __forceinline__ void store_vec(T *__restrict__ p, const T (&s)[VX]) {
  if constexpr (VX * sizeof(T) % 16 == 0) {
    constexpr int E = 16 / sizeof(T);
    using V = __attribute__((ext_vector_type(E))) T;
#pragma unroll
    for (int c = 0; c < VX / E; ++c) {
      V t;
#pragma unroll
      for (int i = 0; i < E; ++i) t[i] = s[c * E + i];
      __builtin_nontemporal_store(t, reinterpret_cast<V *>(p + c * E));
    }
  } else if constexpr (VX * sizeof(T) == 8) {
    using V = __attribute__((ext_vector_type(8 / sizeof(T)))) T;
    V t;
#pragma unroll
    for (int i = 0; i < VX; ++i) t[i] = s[i];
    __builtin_nontemporal_store(t, reinterpret_cast<V *>(p));
  } else {
#pragma unroll
    for (int i = 0; i < VX; ++i) __builtin_nontemporal_store(s[i], p + i);
  }
}

__device__ __forceinline__ int wrap1(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Blocks are dealt round-robin to the 8 XCDs; renumber them so consecutive
// tiles (which share halo rows and columns) run on the same XCD and L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
  if ((nb & 7) != 0) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

}  // namespace k2d
}  // namespace stencil
