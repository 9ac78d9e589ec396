// Conway's Game of Life (one of the paper's Table 1 benchmarks: every cell's
// update depends on its 8 neighbours), one generation per launch on a
// periodic grid of uint8 cells (0 dead, 1 alive).  A cell is alive next iff
// it has exactly 3 live neighbours, or 2 and is alive itself.  The rule is
// not linear, so it is never folded.
//
// One generation per launch (k_life4, k_life1), or several (k_life_tb,
// below).  Rows whose length is a multiple of 4: a thread updates 4 cells
// held in one 32-bit word.  For each of the three rows it loads that word and the two
// bytes beside it; the 3-cell horizontal sums of the 4 cells are formed
// bytewise in one word (each byte stays below 10, so no byte carries into
// the next), and the 8-neighbour count is the three rows' sums minus the
// cell itself.  Other rows: one thread per cell.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>

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

// ---------------------------------------------------------------- K per pass
//
// Several generations per pass over HBM (temporal blocking, as the fused 2D
// sweep): a wavefront streams a 256-cell strip (one 32-bit word of 4 cells
// per lane) down y through K stages; stage s keeps the last two rows of
// generation s it has seen and, when the next row arrives, emits generation
// s+1 of the middle row to stage s+1.  The strip loses one valid cell per
// generation at each end and stores the middle 256 - 2B (B = K rounded up to
// a word); a strip of BY rows streams BY + 2K rows.

// Lane i receives lane i-1's (shr) or lane i+1's (shl) word; end lanes 0.
__device__ __forceinline__ uint32_t word_from_left(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x138, 0xF, 0xF, true);
}
__device__ __forceinline__ uint32_t word_from_right(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x130, 0xF, 0xF, true);
}

// Bytewise: 0x80 in each byte of x that is zero (bytes < 0x80).
__device__ __forceinline__ uint32_t zero_bytes(uint32_t x) {
  return ~((((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x)) & 0x80808080u;
}

// The rule on 4 cells at once: count and self hold one byte per cell.
__device__ __forceinline__ uint32_t rule4_swar(uint32_t self, uint32_t count) {
  const uint32_t eq3 = zero_bytes(count ^ 0x03030303u);
  const uint32_t eq2 = zero_bytes(count ^ 0x02020202u);
  return (eq3 | (eq2 & (self << 7))) >> 7;
}

// 3-cell horizontal sums of the lane's 4 cells (neighbour bytes by DPP).
__device__ __forceinline__ uint32_t hsum(uint32_t w) {
  const uint32_t l = word_from_left(w), r = word_from_right(w);
  return ((w << 8) | (l >> 24)) + w + ((w >> 8) | (r << 24));
}

template <int K>
__global__ void __launch_bounds__(64)
k_life_tb(const uint8_t *__restrict__ in, uint8_t *__restrict__ out, int ny, int nx, int BY,
          int tiles_x) {
  constexpr int B = (K + 3) / 4 * 4;
  constexpr int WOUT = 256 - 2 * B;
  const int lane = threadIdx.x;
  const int t = blockIdx.x;
  const int tx = t % tiles_x, ty = t / tiles_x;
  const int xo0 = tx * WOUT, xi0 = xo0 - B;
  const int y0 = ty * BY, y1 = min(y0 + BY, ny);
  int gx = xi0 + 4 * lane;
  gx = gx < 0 ? gx + nx : (gx >= nx ? gx - nx : gx);
  const int lo = 4 * lane - B;
  const bool store_ok = lo >= 0 && lo + 4 <= WOUT && xo0 + lo + 4 <= nx;
  // per stage a ring of the last three rows of its generation (words and
  // their horizontal sums), rotated by unrolling three rows
  uint32_t rw[K][3], rh[K][3];
#pragma unroll
  for (int s = 0; s < K; ++s)
#pragma unroll
    for (int i = 0; i < 3; ++i) rw[s][i] = rh[s][i] = 0u;
  const int jstart = y0 - K - 1, jend = y1 + K;  // level-0 rows streamed
  auto row_word = [&](int j) {
    j = j < 0 ? j + ny : (j >= ny ? j - ny : j);
    return *reinterpret_cast<const uint32_t *>(in + (size_t)j * nx + gx);
  };
  uint32_t nxt = row_word(jstart);
  for (int jb = jstart; jb < jend; jb += 3) {
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int j = jb + u;
      // rows past jend re-read the last row and are never stored
      uint32_t cur = nxt;
      nxt = row_word(min(j + 1, jend - 1));
      const int a = u % 3, b = (u + 1) % 3, c = (u + 2) % 3;  // prev, mid, incoming
      // stage s: rows (prev, mid, cur) of generation s -> generation s+1 of mid
#pragma unroll
      for (int s = 0; s < K; ++s) {
        const uint32_t hc = hsum(cur);
        const uint32_t next = rule4_swar(rw[s][b], rh[s][a] + rh[s][b] + hc - rw[s][b]);
        rw[s][c] = cur;
        rh[s][c] = hc;
        cur = next;  // generation s+1 of row j - 1 - s
      }
      const int yd = j - K;  // generation K of row yd is complete
      if (store_ok && yd >= y0 && yd < y1)
        *reinterpret_cast<uint32_t *>(out + (size_t)yd * nx + xo0 + lo) = cur;
    }
  }
}

}  // namespace

// Generations one fused launch may take (the launches take 16, 8, 4 or 2);
// 1 when the grid does not suit the fused kernel.
int life_max_steps(int64_t ny, int64_t nx, const void *in, const void *out) {
  if (nx % 4 != 0 || nx < 256 || ny < 33 || (uintptr_t)in % 4 != 0 || (uintptr_t)out % 4 != 0)
    return 1;
  if (nx > (1 << 30) || ny > (1 << 30)) return 1;
  static const int cap = [] {
    const char *e = std::getenv("STENCIL_LIFE_K");
    return e ? std::max(1, std::min(16, std::atoi(e))) : 0;
  }();
  if (cap) return cap;
  // While both grids fit the 256 MB last-level cache, HBM is not the limit
  // and fewer fused generations (less redundant border work) run faster:
  // 4 measured best at 5000^2 (16: -8%); larger grids fuse 16.
  return ny * nx <= (int64_t)(1 << 27) ? 4 : 16;
}

template <int K>
static hipError_t launch_tb(const uint8_t *in, uint8_t *out, int ny, int nx, hipStream_t s) {
  constexpr int WOUT = 256 - 2 * ((K + 3) / 4 * 4);
  const int tiles_x = (nx + WOUT - 1) / WOUT;
  static const int env_by = [] {
    const char *e = std::getenv("STENCIL_LIFE_ROWS");
    return e ? std::atoi(e) : 0;
  }();
  const int target_y = std::max(1, 4096 / tiles_x);
  int by = env_by > 0 ? std::max(env_by, 2 * K) : std::max((ny + target_y - 1) / target_y, 4 * K);
  by = std::min(by, ny);
  const int tiles_y = (ny + by - 1) / by;
  const int64_t blocks = (int64_t)tiles_x * tiles_y;
  if (blocks > (1LL << 31) - 1) return hipErrorNotSupported;
  hipLaunchKernelGGL(k_life_tb<K>, dim3((unsigned)blocks), dim3(64), 0, s, in, out, ny, nx, by,
                     tiles_x);
  return hipGetLastError();
}

hipError_t launch_life_fused(const uint8_t *in, uint8_t *out, int64_t ny, int64_t nx, int K,
                             hipStream_t s) {
  switch (K) {
    case 16: return launch_tb<16>(in, out, (int)ny, (int)nx, s);
    case 8: return launch_tb<8>(in, out, (int)ny, (int)nx, s);
    case 4: return launch_tb<4>(in, out, (int)ny, (int)nx, s);
    case 2: return launch_tb<2>(in, out, (int)ny, (int)nx, s);
    default: return hipErrorNotSupported;
  }
}

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
