// Tiled 3D sweep for gfx950: an (x, y) tile streams through z.
//
// The paper views a 3D grid as a stack of 2D slices (Section 3.3, layout
// preparation); here each workgroup owns a 64 x 16*RY (x, y) tile and a
// segment of z-planes.  Input planes stream through once in ascending z:
//  - each plane of the tile plus an R-wide (x, y) halo (periodic wrap) is
//    staged in a double-buffered LDS slab;
//  - a lane owns 4 consecutive x of RY adjacent rows and keeps the 2R+1
//    output planes a slab contributes to in registers (the accumulator queue
//    along z); each slab row the lane reads serves every one of its rows
//    within R of it; when plane k arrives, output plane k-R is complete and
//    is stored.
// Operation order per output is the canonical one: acc = +0, then one FMA
// per tap of the mask in row-major (oz, oy, ox) order, so results are
// bit-identical to the oracle's FP32 mirror.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <type_traits>

#include "internal.h"

namespace stencil {

namespace {

constexpr int kTX = 16;  // lanes along x
constexpr int kVX = 4;   // points per lane along x
constexpr int kBX = kTX * kVX;
constexpr int kBY = 16;  // rows per tile
constexpr int kThreads = kTX * kBY;

template <typename T, int N>
struct WArr3 {
  T v[N];
};

__device__ __forceinline__ float fma3(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma3(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <int MASK, int R>
__host__ __device__ constexpr bool in_mask3(int oz, int oy, int ox) {
  const int a = oz < 0 ? -oz : oz, b = oy < 0 ? -oy : oy, c = ox < 0 ? -ox : ox;
  return MASK == MASK_BOX ? true
         : MASK == MASK_DIAMOND ? (a + b + c <= R)
                                : ((a != 0) + (b != 0) + (c != 0) <= 1);
}

__device__ __forceinline__ int wrap3(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

template <typename T, int R, int MASK, int RY>
__global__ void __launch_bounds__(kThreads)
k_sweep3d(const T *__restrict__ in, T *__restrict__ out, int nz, int ny, int nx, int BZ,
          int tiles_x, int tiles_y, int vec_ok,
          WArr3<T, (2 * R + 1) * (2 * R + 1) * (2 * R + 1)> W) {
  constexpr int S = 2 * R + 1;
  constexpr int NU = S;
  constexpr int RP = ((R + kVX - 1) / kVX) * kVX;
  constexpr int TBY = kBY * RY;     // tile rows
  constexpr int LW = kBX + 2 * RP;  // slab row width
  constexpr int LH = TBY + 2 * R;   // slab rows
  // halo elements per thread: (LH * (kBX + 2R) - kBX * TBY) / kThreads, rounded up
  constexpr int HN = (LH * (kBX + 2 * R) - kBX * TBY + kThreads - 1) / kThreads;
  __shared__ __attribute__((aligned(32))) T slab[2][LH * LW];

  // consecutive blocks share a z-segment and (x, y)-adjacent tiles; deal
  // them so each XCD gets a contiguous run
  const int nb = gridDim.x;
  const int b = blockIdx.x;
  const int t = (nb & 7) ? b : (b & 7) * (nb >> 3) + (b >> 3);
  const int tx = t % tiles_x;
  const int ty = (t / tiles_x) % tiles_y;
  const int tz = t / (tiles_x * tiles_y);
  const int x0 = tx * kBX, y0 = ty * TBY, z0 = tz * BZ;
  const int w = min(kBX, nx - x0), h = min(TBY, ny - y0);
  const int z1 = min(z0 + BZ, nz);

  const int lane_x = threadIdx.x % kTX, row = (threadIdx.x / kTX) * RY;  // first row
  const int xoff = lane_x * kVX;
  bool valid[RY], full[RY];
#pragma unroll
  for (int ry = 0; ry < RY; ++ry) {
    valid[ry] = (xoff < w) && (row + ry < h);
    full[ry] = valid[ry] && (xoff + kVX <= w) && vec_ok;
  }
  const int xl = x0 + xoff;
  const size_t plane_sz = (size_t)ny * nx;

  // slab[ly * LW + lx] holds (y0 - R + ly, x0 - RP + lx).  Centre points:
  // one vector (or up to kVX scalars) per lane.  Halo points (rows above and
  // below, columns left and right, periodic wrap): a fixed list per lane,
  // computed once; only the plane offset changes from plane to plane.
  size_t c_goff[RY];
  int c_lpos[RY];
#pragma unroll
  for (int ry = 0; ry < RY; ++ry) {
    c_goff[ry] = (size_t)(y0 + row + ry) * nx + xl;
    c_lpos[ry] = (row + ry + R) * LW + RP + xoff;
  }
  size_t h_goff[HN];
  int h_lpos[HN];
  {
    const int lw = w + 2 * R, lh = h + 2 * R;
    const int nh = lw * lh - w * h;
#pragma unroll
    for (int i = 0; i < HN; ++i) {
      const int e = threadIdx.x + i * kThreads;
      h_lpos[i] = -1;
      h_goff[i] = 0;
      if (e < nh) {
        // enumerate the halo ring: top R rows, bottom R rows (full width lw),
        // then the left and right R columns of the h centre rows
        int ly, lxr;
        const int top = R * lw;
        if (e < top) {
          ly = e / lw;
          lxr = e - ly * lw;
        } else if (e < 2 * top) {
          const int f = e - top;
          ly = R + h + f / lw;
          lxr = f % lw;
        } else {
          const int f = e - 2 * top;
          const int r = f / (2 * R), c = f % (2 * R);
          ly = R + r;
          lxr = c < R ? c : w + c;
        }
        const int gy = wrap3(y0 - R + ly, ny);
        const int gx = wrap3(x0 - R + lxr, nx);
        h_goff[i] = (size_t)gy * nx + gx;
        h_lpos[i] = ly * LW + (RP - R + lxr);
      }
    }
  }

  T acc[NU][RY][kVX];
#pragma unroll
  for (int k = 0; k < NU; ++k)
#pragma unroll
    for (int ry = 0; ry < RY; ++ry)
#pragma unroll
      for (int v = 0; v < kVX; ++v) acc[k][ry][v] = T(0);

  // look-ahead ring of NU planes: plane kin sits in slot (kin - kstart) % NU,
  // which is the compile-time index u of the unrolled loop below
  T pc[NU][RY][kVX], ph[NU][HN];
  auto fetch = [&](int kin, T (&c)[RY][kVX], T (&hv)[HN]) {
    const T *plane = in + (size_t)wrap3(kin, nz) * plane_sz;
#pragma unroll
    for (int ry = 0; ry < RY; ++ry) {
      if (full[ry]) {
        using V = __attribute__((ext_vector_type(4))) T;
        V tv = *reinterpret_cast<const V *>(plane + c_goff[ry]);
#pragma unroll
        for (int v = 0; v < kVX; ++v) c[ry][v] = tv[v];
      } else if (valid[ry]) {
#pragma unroll
        for (int v = 0; v < kVX; ++v)
          c[ry][v] = (xoff + v < w) ? plane[c_goff[ry] + v] : T(0);
      }
    }
#pragma unroll
    for (int i = 0; i < HN; ++i)
      if (h_lpos[i] >= 0) hv[i] = plane[h_goff[i]];
  };

  const int kstart = z0 - R, kend = z1 + R;
#pragma unroll
  for (int d = 0; d < NU; ++d)
    if (kstart + d < kend) fetch(kstart + d, pc[d], ph[d]);
  for (int kb = kstart; kb < kend; kb += NU) {
#pragma unroll
    for (int u = 0; u < NU; ++u) {
      const int kin = kb + u;
      if (kin < kend) {
        T *L = slab[(kin - kstart) & 1];
#pragma unroll
        for (int ry = 0; ry < RY; ++ry) {
          if (valid[ry]) {
#pragma unroll
            for (int v = 0; v < kVX; ++v)
              if (full[ry] || xoff + v < w) L[c_lpos[ry] + v] = pc[u][ry][v];
          }
        }
#pragma unroll
        for (int i = 0; i < HN; ++i)
          if (h_lpos[i] >= 0) L[h_lpos[i]] = ph[u][i];
        __syncthreads();
        if (kin + NU < kend) fetch(kin + NU, pc[u], ph[u]);
        // slab rows row - R .. row + RY - 1 + R; row ly serves the lane's
        // rows ry with oy = ly - ry in [-R, R], oy ascending for each ry
#pragma unroll
        for (int ly = -R; ly <= R + RY - 1; ++ly) {
          // aligned reads of the row segment [xoff, xoff + kVX + 2 RP)
          T seg[kVX + 2 * RP];
          const T *src = L + (row + R + ly) * LW + xoff;
#pragma unroll
          for (int i = 0; i < kVX + 2 * RP; i += 4) {
            using V = __attribute__((ext_vector_type(4))) T;
            V tv = *reinterpret_cast<const V *>(src + i);
            seg[i] = tv[0];
            seg[i + 1] = tv[1];
            seg[i + 2] = tv[2];
            seg[i + 3] = tv[3];
          }
#pragma unroll
          for (int ry = 0; ry < RY; ++ry) {
            const int oy = ly - ry;
            if (oy < -R || oy > R) continue;
#pragma unroll
            for (int k = S - 1; k >= 0; --k) {
              const int slot = (u + k) % NU;
              const int oz = R - k;
#pragma unroll
              for (int ox = -R; ox <= R; ++ox) {
                if (in_mask3<MASK, R>(oz, oy, ox)) {
                  const T wt = W.v[((oz + R) * S + (oy + R)) * S + (ox + R)];
#pragma unroll
                  for (int v = 0; v < kVX; ++v)
                    acc[slot][ry][v] = fma3(wt, seg[RP + v + ox], acc[slot][ry][v]);
                }
              }
            }
          }
        }
        // output plane kin - R is complete
        const int zd = kin - R;
#pragma unroll
        for (int ry = 0; ry < RY; ++ry) {
          if (zd >= z0 && valid[ry]) {
            T *dst = out + (size_t)zd * plane_sz + c_goff[ry];
            if (full[ry]) {
              using V = __attribute__((ext_vector_type(4))) T;
              V tv;
#pragma unroll
              for (int v = 0; v < kVX; ++v) tv[v] = acc[u % NU][ry][v];
              __builtin_nontemporal_store(tv, reinterpret_cast<V *>(dst));
            } else {
#pragma unroll
              for (int v = 0; v < kVX; ++v)
                if (xoff + v < w) __builtin_nontemporal_store(acc[u % NU][ry][v], dst + v);
            }
          }
#pragma unroll
          for (int v = 0; v < kVX; ++v) acc[u % NU][ry][v] = T(0);
        }
      }
    }
  }
}

template <typename T, int R, int MASK, int RY>
hipError_t launch_one(const SweepLaunch &L, const std::vector<T> &w) {
  constexpr int S = 2 * R + 1;
  WArr3<T, S * S * S> W;
  for (int i = 0; i < S * S * S; ++i) W.v[i] = w[i];
  const int nz = (int)L.g.nz, ny = (int)L.g.ny, nx = (int)L.g.nx;
  const int tiles_x = (nx + kBX - 1) / kBX, tiles_y = (ny + kBY * RY - 1) / (kBY * RY);
  int bz = 0;
  if (const char *e = std::getenv("STENCIL_TILE_Z")) bz = std::atoi(e);
  if (bz <= 0) {
    const int64_t xy = (int64_t)tiles_x * tiles_y;
    // about 1024 workgroups measured best (128-plane segments at 512^3 with
    // one row per lane), but 512 for two-row tiles at radius 2 (128-plane
    // segments again: a shorter segment repeats more of its 2R-plane halo)
    const int64_t wgs = (RY == 2 && R == 2) ? 512 : 1024;
    const int64_t target_z = std::max<int64_t>(1, (wgs + xy - 1) / xy);
    bz = (int)((nz + target_z - 1) / target_z);
  }
  bz = std::max(bz, std::max(4, 4 * R));
  bz = std::min(bz, nz);
  const int tiles_z = (nz + bz - 1) / bz;
  const int64_t blocks = (int64_t)tiles_x * tiles_y * tiles_z;
  if (blocks > (1LL << 31) - 1) return hipErrorNotSupported;
  // vector loads and stores of kVX elements need kVX-aligned rows and bases
  const int vec_ok = (nx % kVX == 0) && ((uintptr_t)L.in % (kVX * sizeof(T)) == 0) &&
                     ((uintptr_t)L.out % (kVX * sizeof(T)) == 0);
  hipLaunchKernelGGL((k_sweep3d<T, R, MASK, RY>), dim3((unsigned)blocks), dim3(kThreads), 0,
                     L.stream, (const T *)L.in, (T *)L.out, nz, ny, nx, bz, tiles_x, tiles_y,
                     vec_ok, W);
  return hipGetLastError();
}

// Two rows per lane for the FP32 radius-1 box and radius-2 diamond (each
// slab row read serves both rows: for the box 4 row reads per 8 outputs
// instead of 3 per 4; +7% and +3% at 512^3); the 7-point star measured faster
// with one row, and STENCIL_3D_RY = 1 or 2 forces either for FP32 radius 1-2.
template <typename T, int R, int MASK>
hipError_t launch_m(const SweepLaunch &L, const std::vector<T> &w) {
  static const int env = [] {
    const char *e = std::getenv("STENCIL_3D_RY");
    return e ? std::atoi(e) : 0;
  }();
  if constexpr (sizeof(T) == 4 && R <= 2) {
    const bool two = env == 2 || (env != 1 && ((MASK == MASK_BOX && R == 1) ||
                                              (MASK == MASK_DIAMOND && R == 2)));
    if (two) return launch_one<T, R, MASK, 2>(L, w);
  }
  return launch_one<T, R, MASK, 1>(L, w);
}

template <typename T, int R>
hipError_t launch_r(const SweepLaunch &L, const std::vector<T> &w) {
  if (L.op->mask == MASK_BOX) return launch_m<T, R, MASK_BOX>(L, w);
  if (L.op->mask == MASK_AXES && R == 1) return launch_m<T, R, MASK_AXES>(L, w);
  return launch_m<T, R, MASK_DIAMOND>(L, w);  // contains the axes
}

}  // namespace

hipError_t launch_sweep3d(const SweepLaunch &L) {
  if (L.steps != 1) return hipErrorNotSupported;
  if (L.g.nx > (1 << 30) || L.g.ny > (1 << 30) || L.g.nz > (1 << 30))
    return hipErrorNotSupported;
  const int R = L.op->R;
  if (L.dtype == STENCIL_F32) {
    switch (R) {
      case 1: return launch_r<float, 1>(L, L.op->w32);
      case 2: return launch_r<float, 2>(L, L.op->w32);
      case 3: return launch_r<float, 3>(L, L.op->w32);
      default: return hipErrorNotSupported;
    }
  }
  switch (R) {
    case 1: return launch_r<double, 1>(L, L.op->w64);
    case 2: return launch_r<double, 2>(L, L.op->w64);
    default: return hipErrorNotSupported;
  }
}

}  // namespace stencil
