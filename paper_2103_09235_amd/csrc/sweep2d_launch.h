// Host-side launch of one instantiation of the tiled 2D sweep.  Each
// radius is instantiated in its own translation unit (sweep2d_r*.hip) so the
// library builds in parallel.
#pragma once

#include <cstdlib>

#include "sweep2d_impl.h"

namespace stencil {
namespace k2d {

template <typename T, int R, int MASK, int VX, int PD, bool STR, bool SYM = false, int SEPK = 0>
hipError_t launch_one(const SweepLaunch &L, const std::vector<T> &w) {
  constexpr int S = 2 * R + 1;
  constexpr int BX = 64 * VX;
  WArr<T, S * S> W;
  // dense weights, or SEPK pairs of separable factors (2 * SEPK * S < S * S)
  for (int i = 0; i < S * S; ++i) W.v[i] = i < (int)w.size() ? w[i] : T(0);
  const int ny = (int)L.g.ny, nx = (int)L.g.nx;
  const int tiles_x = (nx + BX - 1) / BX;
  int by = 0;
  if (const char *e = std::getenv("STENCIL_TILE_Y")) by = std::atoi(e);
  if (by <= 0) {
    const int target_tiles_y = (4096 + tiles_x - 1) / tiles_x;
    by = (ny + target_tiles_y - 1) / target_tiles_y;
  }
  by = std::max(by, std::max(8, 4 * R));
  by = std::min(by, ny);
  const int tiles_y = (ny + by - 1) / by;
  const int64_t blocks = (int64_t)tiles_x * tiles_y;
  if (blocks > (1LL << 31) - 1) return hipErrorNotSupported;
  // Tile order: for R <= 2 vertically adjacent tiles run together (measured
  // fastest); wider operators order horizontally adjacent tiles together,
  // which cuts the halo-column refetch (FETCH_SIZE -10% at R = 4).
  static const int order_env = [] {
    const char *e = std::getenv("STENCIL_TILE_ORDER");
    return e ? std::atoi(e) : -1;
  }();
  const int xfast = order_env >= 0 ? order_env : (R >= 3 ? 1 : 0);
  hipLaunchKernelGGL((k_sweep2d<T, R, MASK, VX, PD, STR, SYM, SEPK>), dim3((unsigned)blocks), dim3(64), 0,
                     L.stream, (const T *)L.in, (T *)L.out, ny, nx, by, tiles_y, tiles_x,
                     xfast, W);
  return hipGetLastError();
}

template <typename T, int R, int MASK>
hipError_t launch_vx(const SweepLaunch &L, const std::vector<T> &w) {
  constexpr int VXW = 16 / sizeof(T);
  const bool aligned = ((uintptr_t)L.in % 16 == 0) && ((uintptr_t)L.out % 16 == 0) &&
                       (L.g.nx % VXW == 0);
  // rows that are not whole vectors: strided lanes (coalesced scalars)
  if (!aligned) return launch_one<T, R, MASK, VXW, 1, true>(L, w);
  // low-rank operators as sums of separable terms (mode SEPARABLE)
  if constexpr (sizeof(T) == 4) {
    if (L.sep && L.op->sep_rank == 1)
      return launch_one<T, R, MASK_BOX, VXW, 1, false, false, 1>(L, L.op->sep32);
    if (L.sep && L.op->sep_rank == 2 && 4 * (2 * R + 1) < (2 * R + 1) * (2 * R + 1))
      return launch_one<T, R, MASK_BOX, VXW, 1, false, false, 2>(L, L.op->sep32);
  }
  // mirror-symmetric operators may share partial sums (mode SYMMETRIC)
  if (L.sym && L.op->symmetric) {
    if constexpr (R <= 2) return launch_one<T, R, MASK, VXW, 2, false, true>(L, w);
    else return launch_one<T, R, MASK, VXW, 1, false, true>(L, w);
  }
  // (eight columns per lane for the 41-tap fold measured 16% slower than
  // four: the larger register file halves occupancy)
  if constexpr (R <= 2 && rotate_queue<MASK, R, VXW>()) {
    // two rows of look-ahead measured best on gfx950 (STENCIL_PD overrides)
    static const int pd = [] {
      const char *e = std::getenv("STENCIL_PD");
      return e ? std::atoi(e) : 2;
    }();
    if (pd == 2) return launch_one<T, R, MASK, VXW, 2, false>(L, w);
    if (pd == 4) return launch_one<T, R, MASK, VXW, 4, false>(L, w);
  }
  return launch_one<T, R, MASK, VXW, 1, false>(L, w);
}

template <typename T, int R>
hipError_t launch_r(const SweepLaunch &L) {
  const std::vector<T> *w;
  if constexpr (sizeof(T) == 4) w = &L.op->w32;
  else w = &L.op->w64;
  if (L.op->mask == MASK_BOX) return launch_vx<T, R, MASK_BOX>(L, *w);
  return launch_vx<T, R, MASK_DIAMOND>(L, *w);  // the diamond contains the axes
}

}  // namespace k2d
}  // namespace stencil
