// 1D sweep with several time steps fused per launch (temporal blocking in
// registers).
//
// A 1D grid of a few million points is far too small to keep HBM busy for a
// single step (1e6 FP64 points are 16 MB of traffic, about 2 us at HBM
// rate, less than a kernel launch), so one launch advances its block of the
// line k steps: the block loads its 64*4*VX-point span plus k*R halo points
// on each side, every lane keeps VX consecutive points in registers, and
// each step swaps R edge values with the neighbouring lanes through LDS.
// Values near the span's ends go stale by R points per step; the k*R points
// at each end are exactly that stale region and are never stored.  This is
// the GPU counterpart of the paper's tiling in time (Section 3.4, tessellate
// tiling: several steps per tile without reloading), done here with
// overlapping spans instead of triangles, which costs 2kR redundant points
// per span but needs no second phase.
//
// Every step of every point is the plain update in canonical order
// (acc = +0, one FMA per tap, offsets ascending), so results are
// bit-identical to k separate sweeps.
//
// With a floor array (the APOP benchmark of Table 1: option values never
// drop below the exercise payoff) every step ends with u = maxNum(u, floor)
// at each point; the lane keeps its points' floor values in registers.
#include <hip/hip_runtime.h>

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

template <typename T, int R, int VX, bool FLOOR>
__global__ void __launch_bounds__(kThreads)
k_sweep1d(const T *__restrict__ in, T *__restrict__ out, int64_t n, int k,
          int64_t span_out, WArr1<T, 2 * R + 1> W, const T *__restrict__ floor) {
  static_assert(VX >= R, "neighbour values must come from the adjacent lane");
  __shared__ T edge[2][2][kThreads][R];  // [buffer][left/right][lane][i]
  const int t = threadIdx.x;
  const int64_t out0 = (int64_t)blockIdx.x * span_out;  // first output of the block
  const int64_t halo = (int64_t)k * R;
  const int64_t base = out0 - halo + (int64_t)t * VX;    // first point of this lane

  T cur[VX], fl[VX];
#pragma unroll
  for (int v = 0; v < VX; ++v) {
    int64_t g = (base + v) % n;
    if (g < 0) g += n;
    cur[v] = in[g];
    if constexpr (FLOOR) fl[v] = floor[g];
  }

  for (int s = 0; s < k; ++s) {
    const int b = s & 1;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      edge[b][0][t][i] = cur[i];           // my leftmost R values
      edge[b][1][t][i] = cur[VX - R + i];  // my rightmost R values
    }
    __syncthreads();
    T lnb[R], rnb[R];
    const int tl = t > 0 ? t - 1 : t;
    const int tr = t < kThreads - 1 ? t + 1 : t;
#pragma unroll
    for (int i = 0; i < R; ++i) {
      lnb[i] = edge[b][1][tl][i];  // value at position -R + i
      rnb[i] = edge[b][0][tr][i];  // value at position VX + i
    }
    T nxt[VX];
#pragma unroll
    for (int v = 0; v < VX; ++v) {
      T acc = T(0);
#pragma unroll
      for (int o = -R; o <= R; ++o) {
        const int p = v + o;
        const T x = p < 0 ? lnb[R + p] : (p >= VX ? rnb[p - VX] : cur[p]);
        acc = fma1(W.v[o + R], x, acc);
      }
      nxt[v] = FLOOR ? max1(acc, fl[v]) : acc;
    }
#pragma unroll
    for (int v = 0; v < VX; ++v) cur[v] = nxt[v];
  }

#pragma unroll
  for (int v = 0; v < VX; ++v) {
    const int64_t li = (int64_t)t * VX + v;  // index within the loaded span
    if (li >= halo && li < halo + span_out) {
      const int64_t g = out0 + (li - halo);
      if (g < n) out[g] = cur[v];
    }
  }
}

template <typename T>
constexpr int vx_of() {
  return sizeof(T) == 8 ? 16 : 16;
}

template <typename T, int R>
hipError_t launch_r(const SweepLaunch &L, const std::vector<T> &w) {
  constexpr int VX = vx_of<T>();
  WArr1<T, 2 * R + 1> W;
  for (int i = 0; i < 2 * R + 1; ++i) W.v[i] = w[i];
  const int64_t span = (int64_t)kThreads * VX;
  const int64_t span_out = span - 2 * (int64_t)L.steps * R;
  if (span_out < 1) return hipErrorNotSupported;
  const int64_t n = L.g.nx;
  const int64_t blocks = (n + span_out - 1) / span_out;
  if (blocks > (1LL << 31) - 1) return hipErrorNotSupported;
  if (L.floor)
    hipLaunchKernelGGL((k_sweep1d<T, R, VX, true>), dim3((unsigned)blocks), dim3(kThreads), 0,
                       L.stream, (const T *)L.in, (T *)L.out, n, L.steps, span_out, W,
                       (const T *)L.floor);
  else
    hipLaunchKernelGGL((k_sweep1d<T, R, VX, false>), dim3((unsigned)blocks), dim3(kThreads), 0,
                       L.stream, (const T *)L.in, (T *)L.out, n, L.steps, span_out, W,
                       (const T *)nullptr);
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
  // keep the redundant halo work (2kR of 256*16 points) near 5%
  const int64_t span = (int64_t)kThreads * 16;
  return (int)std::max<int64_t>(1, span / (40 * (int64_t)R));
}

hipError_t launch_sweep1d(const SweepLaunch &L) {
  if (L.g.nx > (1LL << 40)) return hipErrorNotSupported;
  if (L.dtype == STENCIL_F32) return launch_t<float>(L, L.op->w32);
  return launch_t<double>(L, L.op->w64);
}

}  // namespace stencil
