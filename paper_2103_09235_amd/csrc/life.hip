// Conway's Game of Life (one of the paper's Table 1 benchmarks: every cell's
// update depends on its 8 neighbours), one generation per launch on a
// periodic grid of uint8 cells (0 dead, 1 alive).  A cell is alive next iff
// it has exactly 3 live neighbours, or 2 and is alive itself.  The rule is
// not linear, so it is never folded.
//
// Rows whose length is a multiple of 4: a thread updates 4 cells held in one
// 32-bit word.  For each of the three rows it loads that word and the two
// bytes beside it; the 3-cell horizontal sums of the 4 cells are formed
// bytewise in one word (each byte stays below 10, so no byte carries into
// the next), and the 8-neighbour count is the three rows' sums minus the
// cell itself.  Other rows: one thread per cell.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace stencil {

namespace {

__device__ __forceinline__ uint32_t rule4(uint32_t self, uint32_t count) {
  uint32_t out = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const uint32_t c = (self >> (8 * j)) & 0xFFu, n = (count >> (8 * j)) & 0xFFu;
    out |= (uint32_t)(n == 3u || (c != 0u && n == 2u)) << (8 * j);
  }
  return out;
}

__global__ void k_life4(const uint8_t *__restrict__ in, uint8_t *__restrict__ out, int64_t ny,
                        int64_t nx) {
  const int64_t wpr = nx / 4;  // words per row
  const int64_t total = ny * wpr;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t y = i / wpr, x0 = (i - y * wpr) * 4;
    const int64_t xl = x0 == 0 ? nx - 1 : x0 - 1;
    const int64_t xr = x0 + 4 == nx ? 0 : x0 + 4;
    uint32_t sum = 0, self = 0;
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      int64_t yy = y + dy;
      yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
      const uint8_t *row = in + yy * nx;
      const uint32_t w = *reinterpret_cast<const uint32_t *>(row + x0);
      const uint32_t left = (w << 8) | row[xl];           // byte j: cell x0 + j - 1
      const uint32_t right = (w >> 8) | ((uint32_t)row[xr] << 24);  // cell x0 + j + 1
      sum += left + w + right;
      if (dy == 0) self = w;
    }
    *reinterpret_cast<uint32_t *>(out + y * nx + x0) = rule4(self, sum - self);
  }
}

__global__ void k_life1(const uint8_t *__restrict__ in, uint8_t *__restrict__ out, int64_t ny,
                        int64_t nx) {
  const int64_t total = ny * nx;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t y = i / nx, x = i - y * nx;
    uint32_t n = 0;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        if (!dy && !dx) continue;
        int64_t yy = y + dy, xx = x + dx;
        yy = yy < 0 ? yy + ny : (yy >= ny ? yy - ny : yy);
        xx = xx < 0 ? xx + nx : (xx >= nx ? xx - nx : xx);
        n += in[yy * nx + xx];
      }
    const uint32_t c = in[i];
    out[i] = (uint8_t)(n == 3u || (c != 0u && n == 2u));
  }
}

}  // namespace

hipError_t launch_life(const uint8_t *in, uint8_t *out, int64_t ny, int64_t nx, hipStream_t s) {
  const bool words = nx % 4 == 0 && (uintptr_t)in % 4 == 0 && (uintptr_t)out % 4 == 0;
  const int64_t work = words ? ny * (nx / 4) : ny * nx;
  const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 1 << 20));
  if (words)
    hipLaunchKernelGGL(k_life4, dim3(blocks), dim3(256), 0, s, in, out, ny, nx);
  else
    hipLaunchKernelGGL(k_life1, dim3(blocks), dim3(256), 0, s, in, out, ny, nx);
  return hipGetLastError();
}

}  // namespace stencil
