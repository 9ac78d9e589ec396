// Separable 3D operators: W[dz][dy][dx] = a[dz] * b[dy] * c[dx], applied as
// three 1D passes in one z-streaming sweep: 3(2R+1) FMAs per point instead of
// the (2R+1)^3 dense taps.  This is the paper's vertical and horizontal
// folding (Section 3.3, Eq. 4-6: the folded unit box is an outer product of
// its column weights and its counterparts) carried to a third axis.
//
// A workgroup owns a 64 x 32 (x, y) tile and a segment of z-planes.  Per
// input plane: the plane (tile plus an R-row and 4-column border, periodic
// wrap) is staged in LDS; the x-pass h = sum_dx c[dx] u[x + dx] runs over the
// tile's rows and the R rows beyond them and goes to LDS; the y-pass
// v = sum_dy b[dy] h[y + dy] then feeds the accumulator queue along z, where
// the 2R+1 pending output planes take a[dz] * v.  Both LDS arrays are
// double-buffered, so a plane costs two barriers.  The summation order
// (x, then y, then z) is not the canonical one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <utility>

#include "internal.h"

namespace stencil {

namespace {

constexpr int kTX = 64, kTY = 32, kThreads = 256;

template <int N>
struct FArr {
  float v[N];
};

__device__ __forceinline__ int wrapn(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

template <typename F, int... Ks>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Ks...>) {
  (f(std::integral_constant<int, Ks>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <int R>
struct SGeo {
  static constexpr int ROWS = kTY + 2 * R;  // rows the x-pass covers
  static constexpr int PW = kTX + 8;        // staged columns: x in [-4, 68)
  static constexpr int PPLANE = ROWS * PW;
  static constexpr int HPLANE = ROWS * kTX;
  static constexpr int NL = (18 * ROWS + kThreads - 1) / kThreads;  // staged runs per thread
  static constexpr int NX = (16 * ROWS + kThreads - 1) / kThreads;  // x-pass runs per thread
  static constexpr int NY = 16 * kTY / kThreads;                    // y-pass runs per thread
};

// V = 4: rows of whole 16-byte vectors (aligned buffers, nx % 4 == 0); 1:
// each column wrapped and stored on its own.
template <int R, int V>
__global__ void __launch_bounds__(kThreads)
k_sweep3d_sep(const float *__restrict__ in, float *__restrict__ out, int nz, int ny, int nx,
              int BZ, int tiles_x, int tiles_y, FArr<3 * (2 * R + 1)> F) {
  static_assert(R >= 1 && R <= 4, "x halo within the 4-column border");
  using G = SGeo<R>;
  constexpr int S = 2 * R + 1;
  constexpr int NU = 2 * S;  // unrolled steps: queue slots and buffer parity
  using V4 = __attribute__((ext_vector_type(4))) float;
  __shared__ __attribute__((aligned(16))) float P[2][G::PPLANE];
  __shared__ __attribute__((aligned(16))) float H[2][G::HPLANE];

  const int nb = gridDim.x, b = blockIdx.x;
  const int t = (nb & 7) ? b : (b & 7) * (nb >> 3) + (b >> 3);  // contiguous per XCD
  const int tx = t % tiles_x, ty = (t / tiles_x) % tiles_y, tz = t / (tiles_x * tiles_y);
  const int x0 = tx * kTX, y0 = ty * kTY, z0 = tz * BZ;
  const int z1 = min(z0 + BZ, nz);
  const int nzs = z1 - z0;
  const int tid = threadIdx.x;
  const size_t plane_sz = (size_t)ny * nx;
  const float *a = F.v, *bw = F.v + S, *c = F.v + 2 * S;

  // staged runs: row r in [0, ROWS) is y0 - R + r, run q in [0, 18) covers
  // x0 - 4 + 4q .. +3
  constexpr int NG = V == 4 ? 1 : 4;
  int soff[G::NL];
  size_t sg[G::NL][NG];
#pragma unroll
  for (int i = 0; i < G::NL; ++i) {
    const int e = tid + kThreads * i;
    soff[i] = e < 18 * G::ROWS ? (e / 18) * G::PW + 4 * (e % 18) : -1;
    const int gy = wrapn(y0 - R + e / 18, ny);
#pragma unroll
    for (int v = 0; v < NG; ++v) sg[i][v] = (size_t)gy * nx + wrapn(x0 - 4 + 4 * (e % 18) + v, nx);
  }
  float pf[2][G::NL][4];
  auto fetch = [&](int j, float(&buf)[G::NL][4]) __attribute__((always_inline)) {
    const float *plane = in + (size_t)wrapn(z0 - R + j, nz) * plane_sz;
#pragma unroll
    for (int i = 0; i < G::NL; ++i) {
      if (soff[i] < 0) continue;
      if constexpr (V == 4) {
        const V4 q = *reinterpret_cast<const V4 *>(plane + sg[i][0]);
        buf[i][0] = q[0]; buf[i][1] = q[1]; buf[i][2] = q[2]; buf[i][3] = q[3];
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) buf[i][v] = plane[sg[i][v]];
      }
    }
  };
  // x-pass runs: row r in [0, ROWS), columns 4q .. 4q+3 of the tile
  int xr[G::NX];
#pragma unroll
  for (int i = 0; i < G::NX; ++i) {
    const int e = tid + kThreads * i;
    xr[i] = e < 16 * G::ROWS ? e : -1;
  }
  // y-pass runs: tile row y in [0, 32), columns 4q .. 4q+3; output offsets
  int yr[G::NY];
  size_t go[G::NY];
  int ok[G::NY];
#pragma unroll
  for (int i = 0; i < G::NY; ++i) {
    const int e = tid + kThreads * i;
    yr[i] = e;
    const int gy = y0 + e / 16, gx = x0 + 4 * (e % 16);
    go[i] = (size_t)gy * nx + gx;
    ok[i] = (gy < ny && gx < nx) ? min(4, nx - gx) : 0;
  }
  float acc[S][G::NY][4];
#pragma unroll
  for (int k = 0; k < S; ++k)
#pragma unroll
    for (int i = 0; i < G::NY; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[k][i][v] = 0.0f;

  fetch(0, pf[0]);
  fetch(1, pf[1]);

  // Step j: input plane j (z = z0 - R + j) contributes to output planes
  // j - R .. j + R (relative), the one at j - R completing (slot j mod S).
  const int J = nzs + 2 * R;
  auto step = [&](auto uc, int j) __attribute__((always_inline)) {
    constexpr int U = decltype(uc)::value;
    constexpr int u = U % S;
    float *Pb = P[U & 1];
    float *Hb = H[U & 1];
#pragma unroll
    for (int i = 0; i < G::NL; ++i)
      if (soff[i] >= 0) {
        V4 q = {pf[U & 1][i][0], pf[U & 1][i][1], pf[U & 1][i][2], pf[U & 1][i][3]};
        *reinterpret_cast<V4 *>(Pb + soff[i]) = q;
      }
    fetch(j + 2, pf[U & 1]);
    __syncthreads();
    // x-pass over the tile's rows and R rows either side
#pragma unroll
    for (int i = 0; i < G::NX; ++i) {
      if (xr[i] < 0) continue;
      const int r = xr[i] / 16, q = xr[i] % 16;
      const float *row = Pb + r * G::PW + 4 * q;  // staged column 4q is x = 4q - 4
      const V4 l4 = *reinterpret_cast<const V4 *>(row);
      const V4 c4 = *reinterpret_cast<const V4 *>(row + 4);
      const V4 r4 = *reinterpret_cast<const V4 *>(row + 8);
      const float seg[12] = {l4[0], l4[1], l4[2], l4[3], c4[0], c4[1], c4[2], c4[3],
                             r4[0], r4[1], r4[2], r4[3]};
      float h[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float s = 0.0f;
#pragma unroll
        for (int dx = -R; dx <= R; ++dx) s = __builtin_fmaf(c[dx + R], seg[4 + v + dx], s);
        h[v] = s;
      }
      V4 hv = {h[0], h[1], h[2], h[3]};
      *reinterpret_cast<V4 *>(Hb + r * kTX + 4 * q) = hv;
    }
    __syncthreads();
    // y-pass, then the z accumulator queue
#pragma unroll
    for (int i = 0; i < G::NY; ++i) {
      const int y = yr[i] / 16, q = yr[i] % 16;
      float vy[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int dy = -R; dy <= R; ++dy) {
        const V4 hv = *reinterpret_cast<const V4 *>(Hb + (y + R + dy) * kTX + 4 * q);
#pragma unroll
        for (int v = 0; v < 4; ++v) vy[v] = __builtin_fmaf(bw[dy + R], hv[v], vy[v]);
      }
#pragma unroll
      for (int k = S - 1; k >= 0; --k) {
        const int slot = (u + k) % S;
        const float wz = a[R - k + R];  // oz = R - k
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[slot][i][v] = __builtin_fmaf(wz, vy[v], acc[slot][i][v]);
      }
    }
    if (j >= 2 * R && j < 2 * R + nzs) {
      float *dst = out + (size_t)(z0 + j - 2 * R) * plane_sz;
#pragma unroll
      for (int i = 0; i < G::NY; ++i) {
        if constexpr (V == 4) {
          if (ok[i] == 4) {
            V4 o = {acc[u][i][0], acc[u][i][1], acc[u][i][2], acc[u][i][3]};
            __builtin_nontemporal_store(o, reinterpret_cast<V4 *>(dst + go[i]));
          }
        } else {
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (v < ok[i]) __builtin_nontemporal_store(acc[u][i][v], dst + go[i] + v);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < G::NY; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[u][i][v] = 0.0f;
  };
  int j0 = 0;
  for (; j0 + NU <= J; j0 += NU)
    static_for<NU>([&](auto k) __attribute__((always_inline)) { step(k, j0 + (int)decltype(k)::value); });
  static_for<NU - 1>([&](auto k) __attribute__((always_inline)) {
    if (j0 + (int)decltype(k)::value < J) step(k, j0 + (int)decltype(k)::value);
  });
}

template <int R, int V>
hipError_t launch_rv(const SweepLaunch &L) {
  constexpr int S = 2 * R + 1;
  FArr<3 * S> F;
  for (int i = 0; i < 3 * S; ++i) F.v[i] = L.op->sep32[i];
  const int nz = (int)L.g.nz, ny = (int)L.g.ny, nx = (int)L.g.nx;
  const int tiles_x = (nx + kTX - 1) / kTX, tiles_y = (ny + kTY - 1) / kTY;
  // about 1024 workgroups; each z-segment repeats 2R planes
  const int64_t xy = (int64_t)tiles_x * tiles_y;
  const int64_t target_z = std::max<int64_t>(1, (1024 + xy - 1) / xy);
  int bz = (int)((nz + target_z - 1) / target_z);
  bz = std::min(std::max(bz, 4 * R), nz);
  const int tiles_z = (nz + bz - 1) / bz;
  const int64_t blocks = xy * tiles_z;
  if (blocks > (1LL << 31) - 1) return hipErrorNotSupported;
  hipLaunchKernelGGL((k_sweep3d_sep<R, V>), dim3((unsigned)blocks), dim3(kThreads), 0, L.stream,
                     (const float *)L.in, (float *)L.out, nz, ny, nx, bz, tiles_x, tiles_y, F);
  return hipGetLastError();
}

template <int R>
hipError_t launch_r(const SweepLaunch &L) {
  const bool vec = L.g.nx % 4 == 0 && (uintptr_t)L.in % 16 == 0 && (uintptr_t)L.out % 16 == 0;
  return vec ? launch_rv<R, 4>(L) : launch_rv<R, 1>(L);
}

}  // namespace

hipError_t launch_sweep3d_sep(const SweepLaunch &L) {
  if (L.steps != 1 || L.dtype != STENCIL_F32 || L.g.dim != 3 || L.op->sep_rank != 1)
    return hipErrorNotSupported;
  if ((int)L.op->sep32.size() != 3 * (2 * L.op->R + 1)) return hipErrorNotSupported;
  if (L.g.nx > (1 << 30) || L.g.ny > (1 << 30) || L.g.nz > (1 << 30) ||
      L.g.nx * L.g.ny > (int64_t)1 << 31)
    return hipErrorNotSupported;
  switch (L.op->R) {
    case 1: return launch_r<1>(L);
    case 2: return launch_r<2>(L);
    case 3: return launch_r<3>(L);
    case 4: return launch_r<4>(L);
    default: return hipErrorNotSupported;
  }
}

}  // namespace stencil
