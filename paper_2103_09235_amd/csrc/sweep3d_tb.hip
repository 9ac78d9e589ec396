// 3D temporal blocking for gfx950: K applications of one operator per pass
// over HBM (the GPU counterpart of the paper's tessellate tiling, Section
// 3.4, which keeps several time steps of a tile in cache between loads).
//
// A workgroup owns a 64 x TY (x, y) output tile and a segment of z-planes,
// and streams the planes through K pipeline stages in ascending z:
//  - level 0 (the input) is staged plane by plane in LDS over the tile plus
//    a border of K*R rows and round4(K*R) columns (periodic wrap), loaded two
//    planes ahead into registers;
//  - stage s (1..K) turns level s-1 into level s over the tile plus the
//    border it still needs ((K-s)*R rows, round4((K-s)*R) columns): each
//    thread owns runs of 4 consecutive x-points and keeps, per run, the 2R+1
//    level-s planes a level-(s-1) plane contributes to in registers (the
//    accumulator queue along z of the single-step kernel); when a plane
//    completes it goes to LDS as stage s+1's input, or to HBM from stage K;
//  - every level's LDS plane is double-buffered and stage s reads the plane
//    stage s-1 wrote in the previous step, so the whole pipeline needs one
//    barrier per input plane.
// Each stored value has gone through K plain applications of the canonical
// chain (acc = +0, one FMA per tap of the mask in row-major (oz, oy, ox)
// order; the overlapped border is recomputed, never exchanged), so the
// result equals K launches of the single-step kernel bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <utility>

#include "internal.h"

namespace stencil {

namespace {

constexpr int kTX = 64;       // output tile width (x)
constexpr int kThreads = 256;

template <int N>
struct WArr {
  float v[N];
};

template <int MASK, int R>
__host__ __device__ constexpr bool in_mask(int oz, int oy, int ox) {
  const int a = oz < 0 ? -oz : oz, b = oy < 0 ? -oy : oy, c = ox < 0 ? -ox : ox;
  return MASK == MASK_BOX ? true
         : MASK == MASK_DIAMOND ? (a + b + c <= R)
                                : ((a != 0) + (b != 0) + (c != 0) <= 1);
}
// some tap of the mask in row oy uses a neighbour column (ox != 0)
template <int MASK, int R>
__host__ __device__ constexpr bool row_needs_x(int oy) {
  for (int oz = -R; oz <= R; ++oz)
    for (int ox = -R; ox <= R; ++ox)
      if (ox != 0 && in_mask<MASK, R>(oz, oy, ox)) return true;
  return false;
}
template <int MASK, int R>
__host__ __device__ constexpr bool row_used(int oy) {
  for (int oz = -R; oz <= R; ++oz)
    for (int ox = -R; ox <= R; ++ox)
      if (in_mask<MASK, R>(oz, oy, ox)) return true;
  return false;
}

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

// Region of level s (0..K): columns [-B(s), 64 + B(s)), rows [-H(s), TY + H(s))
// relative to the tile's first point, in runs of 4 columns.
template <int K, int R, int TY>
struct Geo {
  static constexpr int B(int s) { return ((K - s) * R + 3) / 4 * 4; }
  static constexpr int H(int s) { return (K - s) * R; }
  static constexpr int CW(int s) { return (kTX + 2 * B(s)) / 4; }  // runs per row
  static constexpr int C(int s) { return CW(s) * (TY + 2 * H(s)); }  // runs
  static constexpr int NC(int s) { return (C(s) + kThreads - 1) / kThreads; }
  // LDS plane: level 0's region plus R rows on each side, rows packed with
  // no column margin: consecutive runs of a wavefront that cross to the next
  // row stay 4 columns apart, so a 16-lane group of a 16-byte access never
  // meets the same bank twice (a margin made each such crossing a bank
  // conflict).  The outermost runs of a level s >= 1 read the adjacent row's
  // end instead of a margin: that only reaches columns outside the level's
  // valid width (K-s)R, which B(s) exceeds.
  static constexpr int XOFF = B(0);
  static constexpr int YOFF = H(0) + R;
  static constexpr int LW = kTX + 2 * B(0);
  static constexpr int LH = TY + 2 * H(0) + 2 * R;
  static constexpr int PLANE = LW * LH;
};

// V: 4 = rows of whole 16-byte vectors (nx % 4 == 0, aligned buffers): runs
// are loaded and stored as vectors and never straddle the periodic seam;
// 1 = each column wrapped and stored on its own.
template <int R, int MASK, int K, int TY, int V>
__global__ void __launch_bounds__(kThreads)
k_sweep3d_tb(const float *__restrict__ in, float *__restrict__ out, int nz, int ny, int nx,
             int BZ, int tiles_x, int tiles_y, WArr<(2 * R + 1) * (2 * R + 1) * (2 * R + 1)> W) {
  using G = Geo<K, R, TY>;
  constexpr int S = 2 * R + 1;
  constexpr int NU = 2 * S;  // steps per unrolled round: queue slots and LDS parity
  extern __shared__ __attribute__((aligned(16))) float lds[];  // 2K planes

  const int nb = gridDim.x, b = blockIdx.x;
  const int t = (nb & 7) ? b : (b & 7) * (nb >> 3) + (b >> 3);  // contiguous per XCD
  const int tx = t % tiles_x, ty = (t / tiles_x) % tiles_y, tz = t / (tiles_x * tiles_y);
  const int x0 = tx * kTX, y0 = ty * TY, z0 = tz * BZ;
  const int z1 = min(z0 + BZ, nz);
  const int nzs = z1 - z0;
  const int tid = threadIdx.x;
  const size_t plane_sz = (size_t)ny * nx;

  for (int i = tid; i < 2 * K * G::PLANE; i += kThreads) lds[i] = 0.0f;

  // run slots of each level: LDS offset within a plane (-1 = no run)
  auto run_off = [&](int s, int c) __attribute__((always_inline)) -> int {
    if (c >= G::C(s)) return -1;
    const int cx = c % G::CW(s), cy = c / G::CW(s);
    const int x = -G::B(s) + 4 * cx, y = -G::H(s) + cy;
    return (y + G::YOFF) * G::LW + (x + G::XOFF);
  };
  // level 0: LDS offsets and global offsets within a plane
  constexpr int N0 = G::NC(0);
  constexpr int NG = V == 4 ? 1 : 4;  // global offsets per run: the vector's, or each column's
  int off0[N0];
  size_t g0[N0][NG];
#pragma unroll
  for (int i = 0; i < N0; ++i) {
    const int c = tid + kThreads * i;
    off0[i] = run_off(0, c);
    const int cx = c % G::CW(0), cy = c / G::CW(0);
    const int gy = wrapn(y0 - G::H(0) + cy, ny);
#pragma unroll
    for (int v = 0; v < NG; ++v)
      g0[i][v] = (size_t)gy * nx + wrapn(x0 - G::B(0) + 4 * cx + v, nx);
  }
  // slots past the region re-read the thread's first run (always inside it)
  static_assert(G::C(0) >= kThreads, "every thread owns a level-0 run");
#pragma unroll
  for (int i = 1; i < N0; ++i)
#pragma unroll
    for (int v = 0; v < NG; ++v)
      if (off0[i] < 0) g0[i][v] = g0[0][v];
  float pf[2][N0][4];
  // Every run slot is loaded (slots past the region re-read an in-grid
  // point and are never stored): a load under a branch makes the compiler
  // wait for every access in flight, which would drain the look-ahead.
  auto fetch = [&](int j, float(&buf)[N0][4]) __attribute__((always_inline)) {
    const float *plane = in + (size_t)wrapn(z0 - K * R + j, nz) * plane_sz;
#pragma unroll
    for (int i = 0; i < N0; ++i) {
      if constexpr (V == 4) {
        using V4 = __attribute__((ext_vector_type(4))) float;
        const V4 q = *reinterpret_cast<const V4 *>(plane + g0[i][0]);
        buf[i][0] = q[0]; buf[i][1] = q[1]; buf[i][2] = q[2]; buf[i][3] = q[3];
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) buf[i][v] = plane[g0[i][v]];
      }
    }
  };

  // stage s (1..K): runs, accumulator queues
  constexpr int NCMAX = G::NC(1);
  int offs[K + 1][NCMAX];
#pragma unroll
  for (int s = 1; s <= K; ++s)
#pragma unroll
    for (int i = 0; i < NCMAX; ++i) offs[s][i] = i < G::NC(s) ? run_off(s, tid + kThreads * i) : -1;
  float acc[K + 1][S][NCMAX][4];
#pragma unroll
  for (int s = 0; s <= K; ++s)
#pragma unroll
    for (int k = 0; k < S; ++k)
#pragma unroll
      for (int i = 0; i < NCMAX; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[s][k][i][v] = 0.0f;
  // output runs of stage K: global position, stored if inside the grid
  constexpr int NK = G::NC(K);
  size_t gk[NK];
  int okk[NK];
#pragma unroll
  for (int i = 0; i < NK; ++i) {
    const int c = tid + kThreads * i;
    const int cx = c % G::CW(K), cy = c / G::CW(K);
    const int gx = x0 + 4 * cx, gy = y0 + cy;
    okk[i] = (c < G::C(K) && gy < ny && gx < nx) ? min(4, nx - gx) : 0;
    gk[i] = (size_t)gy * nx + gx;
  }

  fetch(0, pf[0]);
  fetch(1, pf[1]);
  __syncthreads();

  // Step j: level 0 plane j enters LDS; stage s consumes the level-(s-1)
  // plane p = j - 1 - (s-1)(R+1) (written in step j-1) and completes its
  // level-s plane p - R.  Planes are numbered from z0 - K*R; the stored
  // level-K planes are K*R .. K*R + nzs - 1.
  const int J = nzs + K * R + K * (R + 1);
  auto step = [&](auto uc, int j) __attribute__((always_inline)) {
    constexpr int U = decltype(uc)::value;  // j mod NU
    __syncthreads();
    {
      float *L0 = lds + (0 * 2 + (U & 1)) * G::PLANE;
#pragma unroll
      for (int i = 0; i < N0; ++i)
        if (off0[i] >= 0) {
          using V4 = __attribute__((ext_vector_type(4))) float;
          V4 q = {pf[U & 1][i][0], pf[U & 1][i][1], pf[U & 1][i][2], pf[U & 1][i][3]};
          *reinterpret_cast<V4 *>(L0 + off0[i]) = q;
        }
      fetch(j + 2, pf[U & 1]);
    }
    static_for<K>([&](auto sc) __attribute__((always_inline)) {
      constexpr int s = decltype(sc)::value + 1;
      // consumed plane index mod S, and the LDS planes read and written
      constexpr int u = (((U - 1 - (s - 1) * (R + 1)) % S) + S) % S;
      const float *Lin = lds + ((s - 1) * 2 + ((U + 1) & 1)) * G::PLANE;
#pragma unroll
      for (int i = 0; i < G::NC(s); ++i) {
        const int base = offs[s][i];
        if (base < 0) continue;
#pragma unroll
        for (int oy = -R; oy <= R; ++oy) {
          if (!row_used<MASK, R>(oy)) continue;
          using V4 = __attribute__((ext_vector_type(4))) float;
          const float *row = Lin + base + oy * G::LW;
          float seg[12];
          const V4 c4 = *reinterpret_cast<const V4 *>(row);
          seg[4] = c4[0]; seg[5] = c4[1]; seg[6] = c4[2]; seg[7] = c4[3];
          if (row_needs_x<MASK, R>(oy)) {
            const V4 l4 = *reinterpret_cast<const V4 *>(row - 4);
            const V4 r4 = *reinterpret_cast<const V4 *>(row + 4);
            seg[0] = l4[0]; seg[1] = l4[1]; seg[2] = l4[2]; seg[3] = l4[3];
            seg[8] = r4[0]; seg[9] = r4[1]; seg[10] = r4[2]; seg[11] = r4[3];
          }
#pragma unroll
          for (int k = S - 1; k >= 0; --k) {
            const int slot = (u + k) % S;
            const int oz = R - k;
#pragma unroll
            for (int ox = -R; ox <= R; ++ox) {
              if (in_mask<MASK, R>(oz, oy, ox)) {
                const float w = W.v[((oz + R) * S + (oy + R)) * S + (ox + R)];
                // an output plane's first tap (oz = -R, then the lowest oy
                // and ox of that plane's taps) starts its sum from +0, in
                // place of a slot cleared after the plane before
                constexpr int O1 = MASK == MASK_BOX ? -R : 0;
                const bool first = k == S - 1 && oy == O1 && ox == O1;
#pragma unroll
                for (int v = 0; v < 4; ++v)
                  acc[s][slot][i][v] =
                      __builtin_fmaf(w, seg[4 + v + ox], first ? 0.0f : acc[s][slot][i][v]);
              }
            }
          }
        }
      }
      // level-s plane p - R is complete (slot u)
      if constexpr (s < K) {
        float *Lout = lds + (s * 2 + (U & 1)) * G::PLANE;
#pragma unroll
        for (int i = 0; i < G::NC(s); ++i) {
          if (offs[s][i] < 0) continue;
          using V4 = __attribute__((ext_vector_type(4))) float;
          V4 q = {acc[s][u][i][0], acc[s][u][i][1], acc[s][u][i][2], acc[s][u][i][3]};
          *reinterpret_cast<V4 *>(Lout + offs[s][i]) = q;
        }
      } else {
        const int q = j - K * (R + 1);  // level-K plane completed in this step
        if (q >= K * R && q < K * R + nzs) {
          float *dst = out + (size_t)(z0 + q - K * R) * plane_sz;
#pragma unroll
          for (int i = 0; i < NK; ++i) {
            if constexpr (V == 4) {
              if (okk[i] == 4) {
                using V4 = __attribute__((ext_vector_type(4))) float;
                V4 o = {acc[s][u][i][0], acc[s][u][i][1], acc[s][u][i][2], acc[s][u][i][3]};
                __builtin_nontemporal_store(o, reinterpret_cast<V4 *>(dst + gk[i]));
              }
            } else {
#pragma unroll
              for (int v = 0; v < 4; ++v)
                if (v < okk[i]) __builtin_nontemporal_store(acc[s][u][i][v], dst + gk[i] + v);
            }
          }
        }
      }
    });
  };
  // whole rounds of NU steps without a branch, then the last steps
  int j0 = 0;
  for (; j0 + NU <= J; j0 += NU)
    static_for<NU>([&](auto k) __attribute__((always_inline)) { step(k, j0 + (int)decltype(k)::value); });
  static_for<NU - 1>([&](auto k) __attribute__((always_inline)) {
    if (j0 + (int)decltype(k)::value < J) step(k, j0 + (int)decltype(k)::value);
  });
}

template <int R, int MASK, int K, int TY, int V>
hipError_t launch_one(const SweepLaunch &L) {
  using G = Geo<K, R, TY>;
  constexpr int S = 2 * R + 1;
  WArr<S * S * S> W;
  for (int i = 0; i < S * S * S; ++i) W.v[i] = L.op->w32[i];
  const int nz = (int)L.g.nz, ny = (int)L.g.ny, nx = (int)L.g.nx;
  const int tiles_x = (nx + kTX - 1) / kTX, tiles_y = (ny + TY - 1) / TY;
  const size_t lds_bytes = sizeof(float) * 2 * K * G::PLANE;
  static const int env_bz = [] {
    const char *e = std::getenv("STENCIL_TB3_Z");
    return e ? std::atoi(e) : 0;
  }();
  int bz = env_bz;
  if (bz <= 0) {
    // one round: as many workgroups as the CUs' LDS holds at once (each
    // z-segment repeats K*R planes at both ends; at 512^3 the star runs at
    // 1701 GStencil/s so, 1608 with two rounds of half-length segments and
    // 1499 with 256-plane ones; the box at 843, 842 and 595)
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      (void)hipGetLastError();
      cus = 256;
    }
    const int per_cu = std::max<int>(1, (int)(160 * 1024 / lds_bytes));
    const int64_t xy = (int64_t)tiles_x * tiles_y;
    const int64_t target_z = std::max<int64_t>(1, ((int64_t)cus * per_cu + xy - 1) / xy);
    bz = (int)((nz + target_z - 1) / target_z);
  }
  bz = std::max(bz, 2 * K * R);
  bz = std::min(bz, nz);
  const int tiles_z = (nz + bz - 1) / bz;
  const int64_t blocks = (int64_t)tiles_x * tiles_y * tiles_z;
  if (blocks > (1LL << 31) - 1) return hipErrorNotSupported;
  auto kern = k_sweep3d_tb<R, MASK, K, TY, V>;
  static const hipError_t attr = hipFuncSetAttribute(
      reinterpret_cast<const void *>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
      (int)lds_bytes);
  if (attr != hipSuccess) return attr;
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kThreads), lds_bytes, L.stream,
                     (const float *)L.in, (float *)L.out, nz, ny, nx, bz, tiles_x, tiles_y, W);
  return hipGetLastError();
}

template <int R, int MASK, int K, int TY>
hipError_t launch_v(const SweepLaunch &L) {
  const bool vec = L.g.nx % 4 == 0 && (uintptr_t)L.in % 16 == 0 && (uintptr_t)L.out % 16 == 0;
  return vec ? launch_one<R, MASK, K, TY, 4>(L) : launch_one<R, MASK, K, TY, 1>(L);
}

// Most applications one launch fuses, by radius and mask.
int tb3_max(int R, int mask) {
  static const int star_k = [] {
    const char *e = std::getenv("STENCIL_TB3_STAR_K");
    return e ? std::max(1, std::min(4, std::atoi(e))) : 3;
  }();
  if (R == 1) return mask == MASK_BOX ? 2 : star_k;
  // the folded 7-point star (25-point diamond); the folded 27-point box (125
  // taps) is bound by FMA issue already, so fusing it saves nothing
  if (R == 2 && mask != MASK_BOX) return 2;
  return 1;
}

}  // namespace

int sweep3d_max_steps(const SweepLaunch &L) {
  if (L.dtype != STENCIL_F32 || L.g.dim != 3) return 1;
  if (L.g.nx > (1 << 30) || L.g.ny > (1 << 30) || L.g.nz > (1 << 30)) return 1;
  if (L.g.nx * L.g.ny > (int64_t)1 << 31) return 1;
  // at most as many steps as the z-axis holds 2KR+1 planes for
  const int K = std::min<int64_t>(tb3_max(L.op->R, L.op->mask), (L.g.nz - 1) / (2 * L.op->R));
  return std::max(1, K);
}

// Tile heights and depths measured at 512^3 (the alternatives in brackets):
// 7-point star, 3 steps per launch, 16 rows: 1680-1695 GStencil/s (32 rows:
// 1607; 4 steps: 1492, 2 steps: 1188); folded star (25-point diamond), 2
// applications, 16 rows: 1545-1591 (32: 1465); 27-point box, 2 steps, 32
// rows: 840-846 (16: 786).  Taller tiles repeat less border work but hold
// more LDS per workgroup, so fewer workgroups share a CU.
hipError_t launch_sweep3d_tb(const SweepLaunch &L) {
  if (L.steps < 2 || L.steps > sweep3d_max_steps(L)) return hipErrorNotSupported;
  const int R = L.op->R;
  const bool box = L.op->mask == MASK_BOX;
  const bool axes = L.op->mask == MASK_AXES;
  if (R == 1 && box) return L.steps == 2 ? launch_v<1, MASK_BOX, 2, 32>(L) : hipErrorNotSupported;
  if (R == 1) {
    switch (L.steps) {
      case 2: return axes ? launch_v<1, MASK_AXES, 2, 32>(L) : launch_v<1, MASK_DIAMOND, 2, 32>(L);
      case 3: return axes ? launch_v<1, MASK_AXES, 3, 16>(L) : launch_v<1, MASK_DIAMOND, 3, 16>(L);
      case 4: return axes ? launch_v<1, MASK_AXES, 4, 16>(L) : launch_v<1, MASK_DIAMOND, 4, 16>(L);
      default: return hipErrorNotSupported;
    }
  }
  if (R == 2 && L.steps == 2 && !box) return launch_v<2, MASK_DIAMOND, 2, 16>(L);
  return hipErrorNotSupported;
}

}  // namespace stencil
