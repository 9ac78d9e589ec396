// 1D sweep with several time steps fused per launch (temporal blocking in
// registers).
//
// A 1D grid of a few million points is far too small to keep HBM busy for a
// single step (1e6 FP64 points are 16 MB of traffic, about 2 us at HBM
// rate, less than a kernel launch), so one launch advances each span of the
// line k steps: the span's owner loads its points plus k*R halo points on
// each side, every lane keeps VX consecutive points in registers, and each
// step takes R edge values from each neighbouring lane.  Values near the
// span's ends go stale by R points per step; the k*R points at each end are
// exactly that stale region and are never stored.  This is the GPU
// counterpart of the paper's tiling in time (Section 3.4, tessellate tiling:
// several steps per tile without reloading), done here with overlapping
// spans instead of triangles, which costs 2kR redundant points per span but
// needs no second phase.
//
// Two owners of a span:
// * a workgroup of 256 lanes (spans of 256*VX points) exchanging edge values
//   through LDS, one barrier per step: long spans, so few redundant points
//   and many steps per launch, for lines with enough spans to keep several
//   wavefronts on every SIMD, which hide the barrier;
// * a single wavefront (spans of 64*VX points) exchanging edge values with
//   DPP lane shifts, no LDS and no barrier: for short lines (1e6 points fill
//   about one wavefront per SIMD), where every step's LDS round trip and
//   barrier would sit on the critical path of the only wavefront a SIMD has.
//
// Every step of every point is the plain update in canonical order
// (acc = +0, one FMA per tap, offsets ascending), so results are
// bit-identical to k separate sweeps.
//
// With a floor array (the APOP benchmark of Table 1: option values never
// drop below the exercise payoff) every step ends with u = maxNum(u, floor)
// at each point; the lane keeps its points' floor values in registers.
//
// Dirichlet boundaries (a padded line whose interior is [zlo, zhi)): every
// step sets the points outside the interior to the ghost value, their
// indices taken unwrapped, so points past the pad hold it as well, and the
// result is the fixed-ghost sweep at every step.  Spans inside the interior
// skip the test (a uniform branch).
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <type_traits>

#include "internal.h"

namespace stencil {

namespace {

constexpr int kThreads = 256;

template <typename T, int N>
struct WArr1 {
  T v[N];
};

__device__ __forceinline__ float fma1(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma1(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ float max1(float a, float b) { return __builtin_fmaxf(a, b); }
__device__ __forceinline__ double max1(double a, double b) { return __builtin_fmax(a, b); }

// VX consecutive points from index base on (periodic: indices wrap mod n,
// any number of times for a line shorter than the span).
template <typename T, int VX, bool FLOOR>
__device__ __forceinline__ void load_wrapped(const T *__restrict__ in, const T *__restrict__ floor,
                                             int64_t n, int64_t base, T (&cur)[VX],
                                             T (&fl)[VX]) {
  int64_t g = base % n;
  if (g < 0) g += n;
#pragma unroll
  for (int v = 0; v < VX; ++v) {
    cur[v] = in[g];
    if constexpr (FLOOR) fl[v] = floor[g];
    if (++g == n) g = 0;
  }
}

// One step of a lane's VX points (src, with the R values left and right of
// them) into dst.  The step loops alternate two register arrays, two steps
// per iteration, so no step copies its result back.
template <typename T, int R, int VX, bool FLOOR>
__device__ __forceinline__ void step_into(const T (&src)[VX], T (&dst)[VX], const T (&fl)[VX],
                                          const T (&lnb)[R], const T (&rnb)[R],
                                          const WArr1<T, 2 * R + 1> &W) {
#pragma unroll
  for (int v = 0; v < VX; ++v) {
    T acc = T(0);
#pragma unroll
    for (int o = -R; o <= R; ++o) {
      const int p = v + o;
      const T x = p < 0 ? lnb[R + p] : (p >= VX ? rnb[p - VX] : src[p]);
      acc = fma1(W.v[o + R], x, acc);
    }
    dst[v] = FLOOR ? max1(acc, fl[v]) : acc;
  }
}

// Dirichlet: a lane's points (unwrapped indices first .. first+VX-1)
// outside [zlo, zhi) take the ghost value.
template <typename T, int VX>
__device__ __forceinline__ void hold_ghosts(T (&cur)[VX], int64_t first, int64_t zlo, int64_t zhi,
                                            T zval) {
#pragma unroll
  for (int v = 0; v < VX; ++v)
    if (first + v < zlo || first + v >= zhi) cur[v] = zval;
}

// Whole-wavefront DPP shifts by one lane (lane i receives lane i-1's value,
// or lane i+1's; the end lanes receive 0, which lands in the stale halo).
__device__ __forceinline__ int dpp_from_left(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ int dpp_from_right(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x130, 0xF, 0xF, true);
}
__device__ __forceinline__ float from_left(float x) {
  return __builtin_bit_cast(float, dpp_from_left(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ float from_right(float x) {
  return __builtin_bit_cast(float, dpp_from_right(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double from_left(double x) {
  const int2 h = __builtin_bit_cast(int2, x);
  return __builtin_bit_cast(double, make_int2(dpp_from_left(h.x), dpp_from_left(h.y)));
}
__device__ __forceinline__ double from_right(double x) {
  const int2 h = __builtin_bit_cast(int2, x);
  return __builtin_bit_cast(double, make_int2(dpp_from_right(h.x), dpp_from_right(h.y)));
}

// Orders a wavefront's LDS writes before its later reads (lanes of one
// wavefront only; no workgroup barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Index of span point i in a wavefront's LDS tile: one pad slot per 16
// points, so lanes reading 16 consecutive points each (stride 17) hit
// distinct banks.
__device__ __forceinline__ int tile_at(int i) { return i + (i >> 4); }

// A lane's VX consecutive points (from span point lane*VX on) of the
// 64*VX-point span starting at global index base0 (periodic wrap): the
// wavefront reads 64 consecutive points per load instruction into its LDS
// tile, then each lane reads its own points back.
template <typename T, int VX>
__device__ __forceinline__ void gather_span(const T *__restrict__ src, int64_t n, int64_t base0,
                                            int lane, T *tile, T (&dst)[VX]) {
  int64_t g = (base0 + lane) % n;
  if (g < 0) g += n;
#pragma unroll
  for (int v = 0; v < VX; ++v) {
    tile[tile_at(64 * v + lane)] = src[g];
    g += 64;
    while (g >= n) g -= n;
  }
  wave_sync();
#pragma unroll
  for (int v = 0; v < VX; ++v) dst[v] = tile[tile_at(lane * VX + v)];
  wave_sync();
}

// The wavefront-owned span: wavefront wv of the grid owns points
// [wv*span_out, (wv+1)*span_out) and loads 64*VX points from k*R before.
template <typename T, int R, int VX, bool FLOOR>
__global__ void __launch_bounds__(kThreads)
k_sweep1d_wave(const T *__restrict__ in, T *__restrict__ out, int64_t n, int k,
               int64_t span_out, int64_t spans, WArr1<T, 2 * R + 1> W,
               const T *__restrict__ floor, int zb, int64_t zlo, int64_t zhi, T zval) {
  static_assert(VX >= R, "neighbour values must come from the adjacent lane");
  __shared__ T tiles[kThreads / 64][64 * VX + 4 * VX];
  const int lane = threadIdx.x & 63;
  const int64_t wv = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
  if (wv >= spans) return;  // whole wavefronts only; no workgroup barrier below
  T *tile = tiles[threadIdx.x >> 6];
  const int64_t out0 = wv * span_out;
  const int64_t halo = (int64_t)k * R;

  T cur[VX], fl[VX];
  gather_span<T, VX>(in, n, out0 - halo, lane, tile, cur);
  if constexpr (FLOOR) gather_span<T, VX>(floor, n, out0 - halo, lane, tile, fl);
  const int64_t first = out0 - halo + (int64_t)lane * VX;  // unwrapped
  const bool edge_span = zb && (out0 - halo < zlo || out0 - halo + 64 * VX > zhi);
  // the step loop in two versions: spans inside the interior skip the test
  auto steps = [&](auto masked) {
    auto step = [&](const T (&a)[VX], T (&b)[VX]) {
      T lnb[R], rnb[R];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        lnb[i] = from_left(a[VX - R + i]);  // value at position -R + i
        rnb[i] = from_right(a[i]);          // value at position VX + i
      }
      step_into<T, R, VX, FLOOR>(a, b, fl, lnb, rnb, W);
      if constexpr (decltype(masked)::value) hold_ghosts<T, VX>(b, first, zlo, zhi, zval);
    };
    T alt[VX];
    int s = 0;
    for (; s + 2 <= k; s += 2) {
      step(cur, alt);
      step(alt, cur);
    }
    if (s < k) {
      step(cur, alt);
#pragma unroll
      for (int v = 0; v < VX; ++v) cur[v] = alt[v];
    }
  };
  if (edge_span)
    steps(std::true_type{});
  else
    steps(std::false_type{});
  // back through the tile: 64 consecutive points per store instruction
#pragma unroll
  for (int v = 0; v < VX; ++v) tile[tile_at(lane * VX + v)] = cur[v];
  wave_sync();
#pragma unroll
  for (int v = 0; v < VX; ++v) {
    const int i = 64 * v + lane;  // index within the loaded span
    if (i >= halo && i < halo + span_out) {
      const int64_t g = out0 + (i - halo);
      if (g < n) out[g] = tile[tile_at(i)];
    }
  }
}

template <typename T, int R, int VX, bool FLOOR>
__global__ void __launch_bounds__(kThreads)
k_sweep1d(const T *__restrict__ in, T *__restrict__ out, int64_t n, int k,
          int64_t span_out, WArr1<T, 2 * R + 1> W, const T *__restrict__ floor, int zb,
          int64_t zlo, int64_t zhi, T zval) {
  static_assert(VX >= R, "neighbour values must come from the adjacent lane");
  __shared__ T edge[2][2][kThreads][R];  // [buffer][left/right][lane][i]
  const int t = threadIdx.x;
  const int64_t out0 = (int64_t)blockIdx.x * span_out;  // first output of the block
  const int64_t halo = (int64_t)k * R;
  const int64_t base = out0 - halo + (int64_t)t * VX;    // first point of this lane

  T cur[VX], fl[VX];
  load_wrapped<T, VX, FLOOR>(in, floor, n, base, cur, fl);
  const bool edge_span = zb && (out0 - halo < zlo || out0 - halo + kThreads * VX > zhi);

  // step s exchanges edges through buffer s & 1: a buffer is written again
  // only after the next step's barrier, which every reader of it has passed
  const int tl = t > 0 ? t - 1 : t;
  const int tr = t < kThreads - 1 ? t + 1 : t;
  // the step loop in two versions (edge_span is uniform over the block)
  auto steps = [&](auto masked) {
    auto step = [&](const T (&a)[VX], T (&b)[VX], int buf) {
#pragma unroll
      for (int i = 0; i < R; ++i) {
        edge[buf][0][t][i] = a[i];           // my leftmost R values
        edge[buf][1][t][i] = a[VX - R + i];  // my rightmost R values
      }
      __syncthreads();
      T lnb[R], rnb[R];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        lnb[i] = edge[buf][1][tl][i];  // value at position -R + i
        rnb[i] = edge[buf][0][tr][i];  // value at position VX + i
      }
      step_into<T, R, VX, FLOOR>(a, b, fl, lnb, rnb, W);
      if constexpr (decltype(masked)::value) hold_ghosts<T, VX>(b, base, zlo, zhi, zval);
    };
    T alt[VX];
    int s = 0;
    for (; s + 2 <= k; s += 2) {
      step(cur, alt, 0);
      step(alt, cur, 1);
    }
    if (s < k) {
      step(cur, alt, 0);
#pragma unroll
      for (int v = 0; v < VX; ++v) cur[v] = alt[v];
    }
  };
  if (edge_span)
    steps(std::true_type{});
  else
    steps(std::false_type{});

#pragma unroll
  for (int v = 0; v < VX; ++v) {
    const int64_t li = (int64_t)t * VX + v;  // index within the loaded span
    if (li >= halo && li < halo + span_out) {
      const int64_t g = out0 + (li - halo);
      if (g < n) out[g] = cur[v];
    }
  }
}

constexpr int kVX = 16;                        // points per lane
constexpr int64_t kSpanGroup = kThreads * kVX;   // span of the workgroup-owned kernel
constexpr int64_t kSpanWave = 64 * kVX;          // span of the wavefront-owned kernel

// Steps per launch: the workgroup span keeps its redundant halo work (2kR
// of the span) near 5%; the wavefront span allows 10%, since its steps cost
// little beside the launch's own read and write of the line.
int64_t max_steps_for(int64_t span, int R) {
  const int64_t div = span == kSpanWave ? 20 : 40;
  return std::max<int64_t>(1, span / (div * (int64_t)R));
}

// The wavefront-owned kernel while the line has at most about four
// wavefront spans per SIMD (256 CUs x 4 SIMDs); STENCIL_1D_KERNEL=wave or
// group forces one (read once per process).
bool use_wave_kernel(int64_t n, int R) {
  static const int forced = [] {
    const char *e = std::getenv("STENCIL_1D_KERNEL");
    if (!e) return 0;
    if (!std::strcmp(e, "wave")) return 1;
    if (!std::strcmp(e, "group")) return 2;
    return 0;
  }();
  if (forced) return forced == 1;
  const int64_t out = kSpanWave - 2 * max_steps_for(kSpanWave, R) * R;
  return (n + out - 1) / out <= 4 * 1024;
}

// SIMDs of the current device (4 per compute unit), queried once.
int64_t simd_count() {
  static const int64_t simds = [] {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1) {
      (void)hipGetLastError();
      return (int64_t)1024;
    }
    return 4 * (int64_t)cus;
  }();
  return simds;
}

// Points per lane of the wavefront-owned kernel: 8 while 16 would give at
// most two wavefronts per SIMD (the steps of a lone wavefront are bound by
// latency, so twice the wavefronts with half the points each finish sooner
// despite the longer relative halo), else 16.  STENCIL_1D_VX = 8 or 16
// forces one (read once per process).
int wave_vx(int64_t n, int64_t k, int R) {
  static const int forced = [] {
    const char *e = std::getenv("STENCIL_1D_VX");
    const int v = e ? std::atoi(e) : 0;
    return (v == 8 || v == 16) ? v : 0;
  }();
  if (forced) return forced;
  const int64_t out16 = kSpanWave - 2 * k * R;
  const int64_t out8 = kSpanWave / 2 - 2 * k * R;
  if (out8 < 1 || out16 < 1) return 16;
  return (n + out16 - 1) / out16 <= 2 * simd_count() ? 8 : 16;
}

template <typename T, int R>
hipError_t launch_r(const SweepLaunch &L, const std::vector<T> &w) {
  WArr1<T, 2 * R + 1> W;
  for (int i = 0; i < 2 * R + 1; ++i) W.v[i] = w[i];
  const int64_t n = L.g.nx;
  const bool wave = use_wave_kernel(n, R);
  const int vx = wave ? wave_vx(n, L.steps, R) : kVX;
  const int64_t span = wave ? 64 * (int64_t)vx : kSpanGroup;
  const int64_t span_out = span - 2 * (int64_t)L.steps * R;
  if (span_out < 1) return hipErrorNotSupported;
  const int64_t spans = (n + span_out - 1) / span_out;
  const int64_t blocks = wave ? (spans + kThreads / 64 - 1) / (kThreads / 64) : spans;
  if (blocks > (1LL << 31) - 1) return hipErrorNotSupported;
  const T *fl = (const T *)L.floor;
  // Dirichlet: the interior [zlo, zhi) of the padded line, at least R from
  // both ends (the ghosts the first step reads are pad points)
  const int zb = L.zb ? 1 : 0;
  const int64_t zlo = L.zbox[2], zhi = L.zbox[3];
  if (zb && (zlo < R || n - zhi < R || zhi <= zlo)) return hipErrorInvalidValue;
  const T zval = (T)L.zval;
  if (wave && vx == 8) {
    if (fl)
      hipLaunchKernelGGL((k_sweep1d_wave<T, R, 8, true>), dim3((unsigned)blocks), dim3(kThreads),
                         0, L.stream, (const T *)L.in, (T *)L.out, n, L.steps, span_out, spans, W,
                         fl, zb, zlo, zhi, zval);
    else
      hipLaunchKernelGGL((k_sweep1d_wave<T, R, 8, false>), dim3((unsigned)blocks),
                         dim3(kThreads), 0, L.stream, (const T *)L.in, (T *)L.out, n, L.steps,
                         span_out, spans, W, fl, zb, zlo, zhi, zval);
  } else if (wave) {
    if (fl)
      hipLaunchKernelGGL((k_sweep1d_wave<T, R, kVX, true>), dim3((unsigned)blocks),
                         dim3(kThreads), 0, L.stream, (const T *)L.in, (T *)L.out, n, L.steps,
                         span_out, spans, W, fl, zb, zlo, zhi, zval);
    else
      hipLaunchKernelGGL((k_sweep1d_wave<T, R, kVX, false>), dim3((unsigned)blocks),
                         dim3(kThreads), 0, L.stream, (const T *)L.in, (T *)L.out, n, L.steps,
                         span_out, spans, W, fl, zb, zlo, zhi, zval);
  } else if (fl) {
    hipLaunchKernelGGL((k_sweep1d<T, R, kVX, true>), dim3((unsigned)blocks), dim3(kThreads), 0,
                       L.stream, (const T *)L.in, (T *)L.out, n, L.steps, span_out, W, fl, zb,
                       zlo, zhi, zval);
  } else {
    hipLaunchKernelGGL((k_sweep1d<T, R, kVX, false>), dim3((unsigned)blocks), dim3(kThreads), 0,
                       L.stream, (const T *)L.in, (T *)L.out, n, L.steps, span_out, W, fl, zb,
                       zlo, zhi, zval);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_t(const SweepLaunch &L, const std::vector<T> &w) {
  switch (L.op->R) {
    case 1: return launch_r<T, 1>(L, w);
    case 2: return launch_r<T, 2>(L, w);
    case 3: return launch_r<T, 3>(L, w);
    case 4: return launch_r<T, 4>(L, w);
    case 5: return launch_r<T, 5>(L, w);
    case 6: return launch_r<T, 6>(L, w);
    case 7: return launch_r<T, 7>(L, w);
    case 8: return launch_r<T, 8>(L, w);
    default: return hipErrorNotSupported;
  }
}

}  // namespace

int sweep1d_max_steps(const SweepLaunch &L) {
  const int R = L.op->R;
  if (R < 1 || R > 8) return 1;
  return (int)max_steps_for(use_wave_kernel(L.g.nx, R) ? kSpanWave : kSpanGroup, R);
}

hipError_t launch_sweep1d(const SweepLaunch &L) {
  if (L.g.nx > (1LL << 40)) return hipErrorNotSupported;
  if (L.dtype == STENCIL_F32) return launch_t<float>(L, L.op->w32);
  return launch_t<double>(L, L.op->w64);
}

}  // namespace stencil
