// Dirichlet boundaries (every point outside the grid holds a fixed ghost
// value, 0 by default) for plain and folded sweeps.  The paper states no
// boundary; the reading here (with 0; a nonzero ghost value fills the pad
// instead, and the same argument holds since the ghosts keep their value at
// every step):
//
//  * A run works on zero-padded copies of the grid (pad P = m*r on every
//    face of the grid's axes).  Any periodic kernel of the library applied to
//    a padded grid reads zeros where it would read ghosts, so it computes the
//    zero-ghost update at every interior point; the pad points it also writes
//    are cleared again before the next application.
//  * A folded application (Section 3.3: W_m replaces m steps) is exact at
//    points at least (m-1)r from every face: the j-th intermediate point of
//    any path of the m steps it replaces lies within j*r of the output, so no
//    path meets a ghost.  Points in the band closer than (m-1)r take m plain
//    zero-ghost steps instead.  Those are computed on a frame of width
//    2(m-1)r only: level j of the frame is exact closer than 2(m-1)r - (j-1)r
//    to a face (a frame point reads level j-1 within r of itself; level 1
//    reads the complete input), so level m is exact in the band.
//
// The kernels here move boxes between compact and padded arrays, run one
// plain step on the points near the faces (a frame, or the band into the
// application's output) and fill pads with the ghost value.  Each computes
// a point as the canonical chain (acc = +0, one FMA per nonzero tap in
// row-major offset order); a tap that reads the pad adds w*c in its place
// in the chain, and with c = 0 leaves acc unchanged, as dropping it would.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace stencil {

namespace {

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

// Geometry of a padded array: extents np (z, y, x), the interior's first
// index off and extents n per axis.  The grid's own axes have off = P >= 1;
// unit leading axes (dim < 3) have np = n = 1 and off = 0.
struct PadGeom {
  int64_t np[3];
  int64_t off[3];
  int64_t n[3];
};

// The interior points closer than W to a face, as one flat index space so
// that threads share the work evenly: first the "full" rows (row (z, y)
// itself within W of a z or y face) with all nx columns, then every other
// row's two end segments of the x axis.  Along an axis of length n the
// near-face indices are the first and last W (all of them when n <= 2W).
struct Frame {
  int64_t cz, cy;        // near-face counts along z and y (0 on unit axes)
  int64_t nfull, nedge;  // full rows, other rows
  int64_t ea, eb, ecnt;  // x end segments [0, ea) and [eb, nx), ecnt points
  int64_t total;
};

__host__ __device__ inline int64_t near_count(int64_t n, int64_t W, bool axis) {
  return axis ? (n <= 2 * W ? n : 2 * W) : 0;
}
// i-th near-face index along an axis of length n (i < near_count).
__device__ __forceinline__ int64_t near_index(int64_t i, int64_t n, int64_t W) {
  return n <= 2 * W ? i : (i < W ? i : n - 2 * W + i);
}
// i-th index that is not near a face (i < n - near_count).
__device__ __forceinline__ int64_t far_index(int64_t i, int64_t n, int64_t W, bool axis) {
  return axis ? W + i : i;
}

Frame make_frame(const int64_t n[3], const int64_t off[3], int64_t W) {
  Frame f;
  const bool zax = off[0] > 0, yax = off[1] > 0;
  f.cz = near_count(n[0], W, zax);
  f.cy = near_count(n[1], W, yax);
  f.nfull = f.cz * n[1] + (n[0] - f.cz) * f.cy;
  f.nedge = (n[0] - f.cz) * (n[1] - f.cy);
  f.ea = std::min(W, n[2]);
  f.eb = std::max(n[2] - W, f.ea);
  f.ecnt = f.ea + (n[2] - f.eb);
  f.total = f.nfull * n[2] + f.nedge * f.ecnt;
  return f;
}

// Point k of the frame as interior (z, y, x).
__device__ __forceinline__ void frame_point(const PadGeom &g, const Frame &f, int64_t W, int64_t k,
                                            int64_t &z, int64_t &y, int64_t &x) {
  const bool zax = g.off[0] > 0, yax = g.off[1] > 0;
  const int64_t nx = g.n[2], ny = g.n[1], nz = g.n[0];
  if (k < f.nfull * nx) {
    const int64_t row = k / nx;
    x = k - row * nx;
    if (row < f.cz * ny) {
      z = near_index(row / ny, nz, W);
      y = row % ny;
    } else {
      const int64_t r2 = row - f.cz * ny;
      z = far_index(r2 / f.cy, nz, W, zax);
      y = near_index(r2 % f.cy, ny, W);
    }
  } else {
    const int64_t k2 = k - f.nfull * nx;
    const int64_t row = k2 / f.ecnt, i = k2 - row * f.ecnt;
    const int64_t fy = ny - f.cy;
    z = far_index(row / fy, nz, W, zax);
    y = far_index(row % fy, ny, W, yax);
    x = i < f.ea ? i : f.eb + (i - f.ea);
  }
}

// out[z,y,x] (padded, interior coordinates) = one plain application read
// from src (padded).
template <typename T>
__device__ __forceinline__ T apply_at(const T *__restrict__ src, const PadGeom &g, int64_t z,
                                      int64_t y, int64_t x, const int4 *__restrict__ taps,
                                      const T *__restrict__ w, int ntaps) {
  T acc = T(0);
  for (int k = 0; k < ntaps; ++k) {
    const int4 t = taps[k];
    const int64_t zz = z + g.off[0] + t.x, yy = y + g.off[1] + t.y, xx = x + g.off[2] + t.z;
    acc = fma_t(w[t.w], src[(zz * g.np[1] + yy) * g.np[2] + xx], acc);
  }
  return acc;
}

// Copy a box of extents e between arrays with row strides (elements): the
// point (z, y, x) of the box is src[sbase + z*ssz + y*ssy + x] and
// dst[dbase + z*dsz + y*dsy + x].
template <typename T>
__global__ void k_box_copy(const T *__restrict__ src, int64_t sbase, int64_t ssz, int64_t ssy,
                           T *__restrict__ dst, int64_t dbase, int64_t dsz, int64_t dsy,
                           int64_t ez, int64_t ey, int64_t ex) {
  const int64_t N = ez * ey * ex;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < N;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t x = p % ex, q = p / ex, y = q % ey, z = q / ey;
    dst[dbase + z * dsz + y * dsy + x] = src[sbase + z * ssz + y * ssy + x];
  }
}

// One plain step on the frame: every interior point closer than W to a face.
template <typename T>
__global__ void k_frame_step(const T *__restrict__ src, T *__restrict__ dst, PadGeom g, Frame f,
                             int64_t W, const int4 *__restrict__ taps,
                             const T *__restrict__ w, int ntaps) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < f.total;
       k += (int64_t)gridDim.x * blockDim.x) {
    int64_t z, y, x;
    frame_point(g, f, W, k, z, y, x);
    dst[((z + g.off[0]) * g.np[1] + y + g.off[1]) * g.np[2] + x + g.off[2]] =
        apply_at(src, g, z, y, x, taps, w, ntaps);
  }
}

// Set every pad point of a padded array to the ghost value: one wavefront
// per padded row (stores only).
constexpr int kRowsPerBlock = 4;

template <typename T>
__global__ void k_clear_pad(T *__restrict__ dst, PadGeom g, T value) {
  const int64_t prow = (int64_t)blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (prow >= g.np[0] * g.np[1]) return;
  const int64_t py = prow % g.np[1], pz = prow / g.np[1];
  T *d = dst + prow * g.np[2];
  const int64_t z = pz - g.off[0], y = py - g.off[1];
  if (z < 0 || z >= g.n[0] || y < 0 || y >= g.n[1]) {
    for (int64_t px = lane; px < g.np[2]; px += 64) d[px] = value;
    return;
  }
  const int64_t right = g.off[2] + g.n[2];
  const int64_t npad = g.off[2] + (g.np[2] - right);
  for (int64_t i = lane; i < npad; i += 64) d[i < g.off[2] ? i : right + (i - g.off[2])] = value;
}

int blocks_for(int64_t n, int threads) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + threads - 1) / threads, 1 << 20));
}

}  // namespace

// Host helpers used by the Dirichlet run (capi.hip).

hipError_t dirichlet_box_copy(const void *src, int64_t sbase, int64_t ssz, int64_t ssy, void *dst,
                              int64_t dbase, int64_t dsz, int64_t dsy, const int64_t e[3],
                              int dtype, hipStream_t s) {
  const int64_t N = e[0] * e[1] * e[2];
  if (N == 0) return hipSuccess;
  if (dtype == STENCIL_F32)
    hipLaunchKernelGGL(k_box_copy<float>, dim3(blocks_for(N, 256)), dim3(256), 0, s,
                       (const float *)src, sbase, ssz, ssy, (float *)dst, dbase, dsz, dsy, e[0],
                       e[1], e[2]);
  else
    hipLaunchKernelGGL(k_box_copy<double>, dim3(blocks_for(N, 256)), dim3(256), 0, s,
                       (const double *)src, sbase, ssz, ssy, (double *)dst, dbase, dsz, dsy,
                       e[0], e[1], e[2]);
  return hipGetLastError();
}

static PadGeom pad_geom(const int64_t np[3], const int64_t off[3], const int64_t n[3]) {
  PadGeom g;
  for (int a = 0; a < 3; ++a) {
    g.np[a] = np[a];
    g.off[a] = off[a];
    g.n[a] = n[a];
  }
  return g;
}

hipError_t dirichlet_frame_step(const void *src, void *dst, const int64_t np[3],
                                const int64_t off[3], const int64_t n[3], int64_t W,
                                const OperatorDev &op, int dtype, hipStream_t s) {
  const PadGeom g = pad_geom(np, off, n);
  const Frame f = make_frame(n, off, W);
  if (f.total == 0) return hipSuccess;
  const dim3 grid(blocks_for(f.total, 256));
  if (dtype == STENCIL_F32)
    hipLaunchKernelGGL(k_frame_step<float>, grid, dim3(256), 0, s, (const float *)src,
                       (float *)dst, g, f, W, (const int4 *)op.taps_dev,
                       (const float *)op.w_dev, op.ntaps);
  else
    hipLaunchKernelGGL(k_frame_step<double>, grid, dim3(256), 0, s, (const double *)src,
                       (double *)dst, g, f, W, (const int4 *)op.taps_dev,
                       (const double *)op.w_dev, op.ntaps);
  return hipGetLastError();
}

hipError_t dirichlet_clear_pad(void *dst, const int64_t np[3], const int64_t off[3],
                               const int64_t n[3], int dtype, double value, hipStream_t s) {
  const PadGeom g = pad_geom(np, off, n);
  const int64_t blocks = (np[0] * np[1] + kRowsPerBlock - 1) / kRowsPerBlock;
  if (blocks > (1LL << 31) - 1) return hipErrorNotSupported;
  if (dtype == STENCIL_F32)
    hipLaunchKernelGGL(k_clear_pad<float>, dim3((unsigned)blocks), dim3(64 * kRowsPerBlock), 0,
                       s, (float *)dst, g, (float)value);
  else
    hipLaunchKernelGGL(k_clear_pad<double>, dim3((unsigned)blocks), dim3(64 * kRowsPerBlock), 0,
                       s, (double *)dst, g, value);
  return hipGetLastError();
}

}  // namespace stencil
