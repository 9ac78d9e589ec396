// Tiled 2D sweep for gfx950: one wavefront per tile, streaming down y.
//
// One application of a (2R+1)^2 operator (the plain stencil of Section 1, or
// the folded m-step operator of Section 3.3 with R = m*r).  The tile is a
// column strip of 64*VX points (VX consecutive x per lane, loaded as one
// 16-byte vector when VX*sizeof(T) = 16) and BY output rows.  Input rows
// stream through once, top to bottom:
//  - each row (plus R halo columns each side, periodic wrap) is staged in a
//    double-buffered LDS row so a lane can read its neighbours' columns;
//  - the 2R+1 output rows a row contributes to are accumulated in registers
//    (the accumulator queue); when row j arrives, output row j-R completes
//    and is stored, and its registers start output row j+R+1.
// This register reuse along the streaming axis plays the part of the
// paper's shifts reusing (Section 3.4): each input value is loaded from HBM
// once per sweep and read from LDS once per lane that needs it.
//
// Every output keeps the canonical operation order: acc = +0, then one FMA
// per tap of the mask in row-major offset order (rows arrive in ascending
// oy, taps within a row in ascending ox).  Taps inside the mask whose weight
// is zero leave the accumulator unchanged (fma(0, u, acc) == acc for finite
// u and acc != -0), so results are bit-identical to a loop that skips them.
#pragma once

#include <hip/hip_runtime.h>

#include "sweep2d_common.h"

namespace stencil {
namespace k2d {

template <int MASK, int R>
__host__ __device__ constexpr int mask_taps() {
  int n = 0;
  for (int oy = -R; oy <= R; ++oy)
    for (int ox = -R; ox <= R; ++ox) n += in_mask<MASK, R>(oy, ox) ? 1 : 0;
  return n;
}

// Rotating the accumulator queue by unrolling 2R+1 rows avoids register
// moves but multiplies the code size; large operators shift instead.
template <int MASK, int R, int VX>
__host__ __device__ constexpr bool rotate_queue() {
  return (2 * R + 1) * mask_taps<MASK, R>() * VX <= 4096;
}

// LDS row width of a tile routine: 64*VX centre columns plus the halo
// padded to whole vectors.
template <int R, int VX>
__host__ __device__ constexpr int lds_row(int) {
  return 64 * VX + 2 * (((R + VX - 1) / VX) * VX);
}

// One tile: output rows [y0, y1) of the column strip starting at x0, one
// wavefront, streaming input rows y0-R .. y1+R-1.  A lane owns VX columns:
// contiguous ones (STR = false, loaded as one vector; needs rows aligned to
// VX) or the strided columns x0 + lane + 64v (STR = true, one coalesced
// scalar load each; any row length).  Either way 64*VX columns per wave.
// lds: 2 * lds_row<R, VX>() elements of workgroup memory, owned by the caller
// (so several variants in one kernel can share one buffer).
//
// SYM (contiguous lanes only): the operator is symmetric under x -> -x and
// y -> -y, so mirrored inputs are summed once (s_k = u[x-k] + u[x+k]) and each
// input row's partial sum with weight row a feeds both output rows j-a and
// j+a: the counterpart reuse of the paper's vertical and horizontal folding
// (Section 3.3, Eq. 4-6) instead of one FMA per tap.  Fewer operations
// (28 instead of 41 per point for the folded 5-point star at m = 4), but not
// the canonical order.
//
// SEPK > 0 (mode SEPARABLE): the operator is sum_{j<SEPK} a_j b_j^T (W holds
// a_0..a_{SEPK-1}, then b_0..b_{SEPK-1}, S values each) and each input row
// costs 2 * SEPK * S FMAs per point: the horizontal sum h_j = sum_dx
// b_j[dx] u[x+dx], then a_j[oy] * h_j into each pending output row (the
// paper's vertical and horizontal folding of a separable stencil, Eq. 4-6).
template <typename T, int R, int MASK, int VX, int PD, bool STR, bool SYM, typename WA,
          int SEPK = 0>
__device__ __forceinline__ void sweep2d_tile(const T *__restrict__ in, T *__restrict__ out,
                                             int ny, int nx, int x0, int y0, int y1,
                                             const WA &W, T *lds) {
  constexpr int S = 2 * R + 1;
  constexpr int NU = S;
  // the separable form's rows are short enough to unroll a whole queue turn
  constexpr bool ROT = SEPK > 0 || rotate_queue<MASK, R, VX>();
  static_assert(ROT || PD == 1, "look-ahead needs the rotating queue");
  constexpr int UNR = ROT ? NU * PD : 1;
  constexpr int BX = 64 * VX;
  constexpr int RP = ((R + VX - 1) / VX) * VX;
  constexpr int LW = BX + 2 * RP;
  static_assert(LW == lds_row<R, VX>(0), "lds row");

  const int lane = threadIdx.x;
  const int w = min(BX, nx - x0);
  // local column of element v and whether it lies inside the strip
  auto col = [&](int v) { return STR ? lane + 64 * v : lane * VX + v; };
  bool ok[VX];
#pragma unroll
  for (int v = 0; v < VX; ++v) ok[v] = col(v) < w;
  const bool valid = ok[0];
  const int xl = x0 + lane * VX;
  __syncthreads();  // a previous tile of this wavefront may still own the rows

  int hx = -1, hpos = 0;
  if (lane < R) {
    hx = wrap1(x0 - R + lane, nx);
    hpos = RP - R + lane;
  } else if (lane < 2 * R) {
    hx = wrap1(x0 + w + lane - R, nx);
    hpos = RP + w + lane - R;
  }

  T acc[NU][VX];
#pragma unroll
  for (int k = 0; k < NU; ++k)
#pragma unroll
    for (int v = 0; v < VX; ++v) acc[k][v] = T(0);

  const int jstart = y0 - R, jend = y1 + R;

  auto load_row = [&](const T *row, T (&d)[VX]) {
    if constexpr (STR) {
#pragma unroll
      for (int v = 0; v < VX; ++v)
        if (ok[v]) d[v] = __builtin_nontemporal_load(row + x0 + col(v));
    } else {
      if (valid) load_vec<T, VX>(row + xl, d);
    }
  };

  // ring of PD rows of look-ahead (centre values + halo element); row j
  // sits in slot (j - jstart) % PD, a compile-time index in the unrolled loop
  T pf[PD][VX];
  T pfh[PD];
#pragma unroll
  for (int d = 0; d < PD; ++d) {
    pfh[d] = T(0);
#pragma unroll
    for (int v = 0; v < VX; ++v) pf[d][v] = T(0);
    if (jstart + d < jend) {
      const T *row = in + (size_t)wrap1(jstart + d, ny) * nx;
      load_row(row, pf[d]);
      if (hx >= 0) pfh[d] = row[hx];
    }
  }

  for (int jb = jstart; jb < jend; jb += UNR) {
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int j = jb + u;
      if (j < jend) {
        T cur[VX];
#pragma unroll
        for (int v = 0; v < VX; ++v) cur[v] = pf[u % PD][v];
        const T curh = pfh[u % PD];
        if (j + PD < jend) {
          const T *row = in + (size_t)wrap1(j + PD, ny) * nx;
          load_row(row, pf[u % PD]);
          if (hx >= 0) pfh[u % PD] = row[hx];
        }
        T *L = lds + ((j - jstart) & 1) * LW;
        if constexpr (STR) {
#pragma unroll
          for (int v = 0; v < VX; ++v)
            if (ok[v]) L[RP + col(v)] = cur[v];
        } else {
          if (valid) store_vec<T, VX>(L + RP + lane * VX, cur);
        }
        if (hx >= 0) L[hpos] = curh;
        __syncthreads();
        // win[v][ox + R] = value at column col(v) + ox (strided), or
        // win[0][i] = value at x = xl + i - RP (contiguous)
        constexpr int WN = STR ? S : VX + 2 * RP;
        constexpr int WV = STR ? VX : 1;
        T win[WV][WN];
        if constexpr (STR) {
#pragma unroll
          for (int v = 0; v < VX; ++v)
#pragma unroll
            for (int i = 0; i < S; ++i)
              win[v][i] = (i == R) ? cur[v] : L[RP + col(v) + i - R];
        } else {
#pragma unroll
          for (int i = 0; i < RP; ++i) win[0][i] = (i >= RP - R) ? L[lane * VX + i] : T(0);
#pragma unroll
          for (int v = 0; v < VX; ++v) win[0][RP + v] = cur[v];
#pragma unroll
          for (int i = RP + VX; i < VX + 2 * RP; ++i)
            win[0][i] = (i < RP + VX + R) ? L[lane * VX + i] : T(0);
        }
        if constexpr (SEPK > 0) {
          static_assert(!STR && !SYM, "separable rows use contiguous lanes");
#pragma unroll
          for (int jr = 0; jr < SEPK; ++jr) {
            T h[VX];
#pragma unroll
            for (int ox = -R; ox <= R; ++ox) {
              const T bt = W[(SEPK + jr) * S + ox + R];
#pragma unroll
              for (int v = 0; v < VX; ++v)
                h[v] = fmat(bt, win[0][RP + v + ox], ox == -R ? T(0) : h[v]);
            }
#pragma unroll
            for (int k = S - 1; k >= 0; --k) {
              const int slot = (u + k) % NU;
              const T at = W[jr * S + (R - k) + R];
#pragma unroll
              for (int v = 0; v < VX; ++v) acc[slot][v] = fmat(at, h[v], acc[slot][v]);
            }
          }
        } else if constexpr (SYM) {
          static_assert(!STR, "shared partial sums use contiguous lanes");
          // sp[k][v] = u[x+k] + u[x-k] (sp[0] = u[x]) for the lane's columns
          T sp[R + 1][VX];
#pragma unroll
          for (int v = 0; v < VX; ++v) {
            sp[0][v] = win[0][RP + v];
#pragma unroll
            for (int k = 1; k <= R; ++k) sp[k][v] = win[0][RP + v - k] + win[0][RP + v + k];
          }
#pragma unroll
          for (int a = 0; a <= R; ++a) {
            // weight row a (= row -a): h = sum_k W[a][k] * sp[k]
            T h[VX];
#pragma unroll
            for (int k = 0; k <= R; ++k) {
              if (in_mask<MASK, R>(a, k)) {
                const T wt = W[(a + R) * S + (k + R)];
#pragma unroll
                for (int v = 0; v < VX; ++v) h[v] = (k == 0) ? wt * sp[0][v] : fmat(wt, sp[k][v], h[v]);
              }
            }
            // input row j feeds output row j - oy through weight row oy;
            // the pending row for oy sits at queue index R - oy
            const int s1 = ROT ? (u + R - a) % NU : R - a;
#pragma unroll
            for (int v = 0; v < VX; ++v) acc[s1][v] += h[v];
            if (a > 0) {
              const int s2 = ROT ? (u + R + a) % NU : R + a;
#pragma unroll
              for (int v = 0; v < VX; ++v) acc[s2][v] += h[v];
            }
          }
        } else {
#pragma unroll
        for (int k = S - 1; k >= 0; --k) {
          // pending output row y = j - R + k receives weight row oy = R - k
          // (rows outside [y0, y1) accumulate too and are simply never
          // stored: cheaper than a branch per pending row)
          const int slot = ROT ? (u + k) % NU : k;
          const int oy = R - k;
#pragma unroll
          for (int ox = -R; ox <= R; ++ox) {
            if (in_mask<MASK, R>(oy, ox)) {
              const T wt = W[(oy + R) * S + (ox + R)];
#pragma unroll
              for (int v = 0; v < VX; ++v)
                acc[slot][v] = fmat(wt, STR ? win[v % WV][ox + R] : win[0][RP + v + ox], acc[slot][v]);
            }
          }
        }
        }
        // output row j - R is complete
        const int yd = j - R;
        T(&done)[VX] = acc[ROT ? u % NU : 0];
        if (yd >= y0) {
          T *dst = out + (size_t)yd * nx;
          if constexpr (STR) {
#pragma unroll
            for (int v = 0; v < VX; ++v)
              if (ok[v]) __builtin_nontemporal_store(done[v], dst + x0 + col(v));
          } else {
            if (valid) store_vec<T, VX>(dst + xl, done);
          }
        }
        if constexpr (ROT) {
#pragma unroll
          for (int v = 0; v < VX; ++v) acc[u % NU][v] = T(0);
        } else {
#pragma unroll
          for (int k = 0; k + 1 < NU; ++k)
#pragma unroll
            for (int v = 0; v < VX; ++v) acc[k][v] = acc[k + 1][v];
#pragma unroll
          for (int v = 0; v < VX; ++v) acc[NU - 1][v] = T(0);
        }
      }
    }
  }
}

template <typename T, int R, int MASK, int VX, int PD, bool STR, bool SYM, int SEPK = 0>
__global__ void __launch_bounds__(64)
k_sweep2d(const T *__restrict__ in, T *__restrict__ out, int ny, int nx, int BY,
          int tiles_y, int tiles_x, int xfast, WArr<T, (2 * R + 1) * (2 * R + 1)> W) {
  constexpr int BX = 64 * VX;
  const int t = xcd_tile(blockIdx.x, gridDim.x);
  // xfast: horizontally adjacent tiles are consecutive (they run together
  // and share halo columns through L2); else vertically adjacent ones are.
  const int tx = xfast ? t % tiles_x : t / tiles_y;
  const int ty = xfast ? t / tiles_x : t - tx * tiles_y;
  const int x0 = tx * BX, y0 = ty * BY;
  const int y1 = min(y0 + BY, ny);
  __shared__ T lds[2 * lds_row<R, VX>(0)];
  sweep2d_tile<T, R, MASK, VX, PD, STR, SYM, WArr<T, (2 * R + 1) * (2 * R + 1)>, SEPK>(
      in, out, ny, nx, x0, y0, y1, W, lds);
}

}  // namespace k2d
}  // namespace stencil
