// Folded 2D stencil as banded-Toeplitz matrix products on the gfx950 matrix
// cores (v_mfma_f32_16x16x32_bf16), with BF16 hi+lo splitting of both
// operands and FP32 accumulation.
//
// Folding m steps (Section 3.3) turns a 3x3 box into a dense (2R+1)^2 box,
// R = m*r, dense enough that one output tile is a sum of matrix products:
//   out[y0+i][x0+n] = sum_dy sum_k A_dy[i][k] * B_dy[k][n],
//   A_dy[i][k] = u[y0+i+dy][x0-R+k]           (16 x 32, rows of the input),
//   B_dy[k][n] = W[dy][k-n-R] if |k-n-R| <= R  (32 x 16, banded Toeplitz),
// with K = 32 >= 16 + 2R for R <= 8.  Each operand is split into
// bf16 hi = bf16(x) and lo = bf16(x - hi); three products (hi*hi, hi*lo,
// lo*hi) recover about 16 significant bits, so the result stays within 1e-3
// of the FP64 sweep over hundreds of folded steps, unlike a single BF16
// product.  Unlike the vector kernels this form does not keep the canonical
// summation order: the matrix unit adds in its own order.
//
// Work layout: a workgroup of 4 wavefronts owns a 128-column strip of a
// segment of rows; wavefront w computes two 16-column blocks.  Input rows are
// staged 16 at a time into an LDS ring (64 rows, split into hi and lo planes)
// one chunk ahead of the products; the B_dy fragments (hi and lo) stay in
// registers for the whole kernel, loaded from a table the host builds once
// per operator.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>

#include "internal.h"

namespace stencil {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kBlocks = 2;                     // 16-column blocks per wavefront
constexpr int kStrip = 16 * kWaves * kBlocks;  // output columns per workgroup
constexpr int kRing = 64;            // staged rows: 4 chunks of 16 (3 in use)

__device__ __forceinline__ unsigned short bf16_bits_rne(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ int wrapfull(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// VEC: rows hold a multiple of 4 floats and the input is 16-byte aligned, so
// staging reads aligned float4 groups (a group never straddles the periodic
// seam); otherwise one float at a time.
template <int R, bool VEC>
__global__ void __launch_bounds__(kThreads)
k_mfma2d(const float *__restrict__ in, float *__restrict__ out, int ny, int nx, int rows_per_wg,
         int tiles_x, const uint4 *__restrict__ btab) {
  static_assert(R >= 1 && R <= 8, "K = 32 covers 16 + 2R columns for R <= 8");
  constexpr int S = 2 * R + 1;
  constexpr int SW = kStrip + 2 * R;  // staged columns: x = x0 - R + c
  // an A fragment spans 32 columns from its block's first column, so ring
  // rows hold kStrip + 16 columns; those past the staged width are zero
  // (finite, and multiplied by zero weights)
  constexpr int SWP = kStrip + 16;
  static_assert(SW <= SWP, "staged width");
  // staging work per thread per chunk of 16 rows
  constexpr int NG = SWP / 4;                              // float4 groups per row
  constexpr int PERV = (16 * NG + kThreads - 1) / kThreads;
  constexpr int PERS = (16 * SW + kThreads - 1) / kThreads;
  constexpr int PER = VEC ? PERV : PERS;
  __shared__ __attribute__((aligned(16))) unsigned short s_hi[kRing][SWP];
  __shared__ __attribute__((aligned(16))) unsigned short s_lo[kRing][SWP];
  __shared__ __attribute__((aligned(16))) float s_out[16][kStrip + 4];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lg = lane >> 4;
  const int tile = blockIdx.x;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int x0 = tx * kStrip;
  const int ybase = ty * rows_per_wg;
  const int yend = min(ybase + rows_per_wg, ny);
  const int nchunks = (yend - ybase + 15) / 16;

  // B_dy fragments (lane (n = li, g = lg) holds k = 8g + j), built once on
  // the host: btab[(2d) * 64 + lane] = hi, btab[(2d + 1) * 64 + lane] = lo
  bf16x8 bhi[S], blo[S];
#pragma unroll
  for (int d = 0; d < S; ++d) {
    bhi[d] = __builtin_bit_cast(bf16x8, btab[(2 * d) * 64 + lane]);
    blo[d] = __builtin_bit_cast(bf16x8, btab[(2 * d + 1) * 64 + lane]);
  }

  // staging step s covers input rows ybase - R + 16s + [0, 16), ring slots
  // 16*(s % 4) + [0, 16).  A thread stages the same (row, column group)
  // pairs at every step, so their wrapped columns are computed once; rows
  // and columns use a full modulo because the staged window may exceed a
  // small grid several times over.
  f32x4 pv[PER];
  int prow[PER], pgx[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = tid + p * kThreads;
    prow[p] = -1;
    pgx[p] = 0;
    if (VEC ? e < 16 * NG : e < 16 * SW) {
      const int per_row = VEC ? NG : SW;
      const int r = e / per_row, q = e - r * per_row;
      prow[p] = r;
      // VEC: group q covers x = x0 - 8 + 4q .. +3 (aligned, never split by
      // the seam since nx % 4 == 0); else column q is x = x0 - R + q
      pgx[p] = wrapfull(VEC ? x0 - 8 + 4 * q : x0 - R + q, nx);
    }
  }
  auto fetch = [&](int s) {
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      if (prow[p] >= 0) {
        const int gy = wrapfull(ybase - R + 16 * s + prow[p], ny);
        const float *src = in + (size_t)gy * nx + pgx[p];
        if constexpr (VEC)
          pv[p] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(src));
        else
          pv[p][0] = __builtin_nontemporal_load(src);
      }
    }
  };
  // hi = bf16(x), lo = bf16(x - hi), both rounded to nearest even (the
  // hardware conversion on gfx950)
  auto split = [](float x, unsigned short &h, unsigned short &l) {
    const __bf16 hb = (__bf16)x;
    const __bf16 lb = (__bf16)(x - (float)hb);
    h = __builtin_bit_cast(unsigned short, hb);
    l = __builtin_bit_cast(unsigned short, lb);
  };
  auto stage = [&](int s) {
    const int slot0 = 16 * (s & 3);
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      if (prow[p] < 0) continue;
      const int r = prow[p];
      if constexpr (VEC) {
        const int e = tid + p * kThreads;
        const int q = e - r * NG;
        const int c0 = 4 * q - 8 + R;  // staged column of the group's first value
        unsigned short h[4], l[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) split(pv[p][t], h[t], l[t]);
        if constexpr (R % 4 == 0) {
          // c0 is a multiple of 4: one 8-byte store per plane
          if (c0 >= 0 && c0 + 4 <= SW) {
            uint2 hv = {(unsigned)h[0] | ((unsigned)h[1] << 16), (unsigned)h[2] | ((unsigned)h[3] << 16)};
            uint2 lv = {(unsigned)l[0] | ((unsigned)l[1] << 16), (unsigned)l[2] | ((unsigned)l[3] << 16)};
            *reinterpret_cast<uint2 *>(&s_hi[slot0 + r][c0]) = hv;
            *reinterpret_cast<uint2 *>(&s_lo[slot0 + r][c0]) = lv;
          }
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (c0 + t >= 0 && c0 + t < SW) {
              s_hi[slot0 + r][c0 + t] = h[t];
              s_lo[slot0 + r][c0 + t] = l[t];
            }
        }
      } else {
        const int e = tid + p * kThreads;
        const int c = e - r * SW;
        unsigned short h, l;
        split(pv[p][0], h, l);
        s_hi[slot0 + r][c] = h;
        s_lo[slot0 + r][c] = l;
      }
    }
  };

  for (int e = tid; e < kRing * (SWP - SW); e += kThreads) {
    const int r = e / (SWP - SW), c = SW + e % (SWP - SW);
    s_hi[r][c] = 0;
    s_lo[r][c] = 0;
  }
  fetch(0);
  stage(0);
  fetch(1);
  stage(1);
  __syncthreads();

  for (int c = 0; c < nchunks; ++c) {
    const bool more = c + 2 <= nchunks;  // chunk c+1 will need staging step c+2
    if (more) fetch(c + 2);
    // three independent accumulation chains per block (one per product
    // kind) keep the matrix pipe busy; the two small ones are added first
    f32x4 acc_lh[kBlocks], acc_hl[kBlocks], acc_hh[kBlocks];
    // A fragments at step d: lane (i, g) of block b needs staged row
    // 16c + i + d, columns cb + 8g .. cb + 8g + 7, read from LDS (hi and lo).
    // (Carrying the lo plane in registers and moving it one row per step
    // with DPP row_shl/row_ror was measured slower: the moves cost more
    // VALU issue than the LDS reads they save.)
#pragma unroll
    for (int b = 0; b < kBlocks; ++b) acc_lh[b] = acc_hl[b] = acc_hh[b] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int d = 0; d < S; ++d) {
      const int slot = (16 * c + li + d) & (kRing - 1);
#pragma unroll
      for (int b = 0; b < kBlocks; ++b) {
        const int col = 16 * (kBlocks * wave + b) + 8 * lg;
        const bf16x8 h = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(&s_hi[slot][col]));
        const bf16x8 l = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(&s_lo[slot][col]));
        acc_lh[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(l, bhi[d], acc_lh[b], 0, 0, 0);
        acc_hl[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, blo[d], acc_hl[b], 0, 0, 0);
        acc_hh[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(h, bhi[d], acc_hh[b], 0, 0, 0);
      }
    }
    // D fragment: lane holds column li, rows 4*lg + j.  The workgroup's
    // 16 x kStrip output tile goes through LDS so that rows leave as whole
    // 16-byte groups (scattered 4-byte stores of 16-lane rows cost about a
    // third more HBM write traffic).
#pragma unroll
    for (int b = 0; b < kBlocks; ++b) {
      const int oc = 16 * (kBlocks * wave + b) + li;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        s_out[4 * lg + j][oc] = (acc_lh[b][j] + acc_hl[b][j]) + acc_hh[b][j];
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < (16 * kStrip / 4) / kThreads; ++p) {
      const int e = tid + p * kThreads;
      const int r = e / (kStrip / 4), q = e - r * (kStrip / 4);
      const int yo = ybase + 16 * c + r, xo = x0 + 4 * q;
      if (yo < yend) {
        float *dst = out + (size_t)yo * nx + xo;
        const f32x4 v = *reinterpret_cast<const f32x4 *>(&s_out[r][4 * q]);
        if (VEC && xo + 4 <= nx) {
          __builtin_nontemporal_store(v, reinterpret_cast<f32x4 *>(dst));
        } else {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (xo + t < nx) __builtin_nontemporal_store(v[t], dst + t);
        }
      }
    }
    if (more) stage(c + 2);
    __syncthreads();
  }
}

template <int R>
hipError_t launch_r(const SweepLaunch &L) {
  const int ny = (int)L.g.ny, nx = (int)L.g.nx;
  const int tiles_x = (nx + kStrip - 1) / kStrip;
  int rows = 0;
  if (const char *e = std::getenv("STENCIL_MFMA_ROWS")) rows = std::atoi(e);
  if (rows <= 0) {
    const int target_y = std::max(1, (4096 + tiles_x - 1) / tiles_x);
    rows = (ny + target_y - 1) / target_y;
  }
  rows = std::max(32, (rows + 15) / 16 * 16);
  const int tiles_y = (ny + rows - 1) / rows;
  const int64_t blocks = (int64_t)tiles_x * tiles_y;
  if (blocks > (1LL << 31) - 1 || !L.op->mfma_b) return hipErrorNotSupported;
  const bool vec = (nx % 4 == 0) && ((uintptr_t)L.in % 16 == 0) && ((uintptr_t)L.out % 16 == 0);
  const uint4 *bt = (const uint4 *)L.op->mfma_b;
  const dim3 grid((unsigned)blocks), blk(kThreads);
  if (vec)
    hipLaunchKernelGGL((k_mfma2d<R, true>), grid, blk, 0, L.stream, (const float *)L.in,
                       (float *)L.out, ny, nx, rows, tiles_x, bt);
  else
    hipLaunchKernelGGL((k_mfma2d<R, false>), grid, blk, 0, L.stream, (const float *)L.in,
                       (float *)L.out, ny, nx, rows, tiles_x, bt);
  return hipGetLastError();
}

uint16_t bf16_host(float x) {
  uint32_t b;
  std::memcpy(&b, &x, 4);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

}  // namespace

hipError_t launch_mfma2d(const SweepLaunch &L) {
  if (L.steps != 1 || L.dtype != STENCIL_F32 || L.g.dim != 2) return hipErrorNotSupported;
  if (L.g.ny > (1 << 30) || L.g.nx > (1 << 30)) return hipErrorNotSupported;
  switch (L.op->R) {
    case 1: return launch_r<1>(L);
    case 2: return launch_r<2>(L);
    case 3: return launch_r<3>(L);
    case 4: return launch_r<4>(L);
    case 5: return launch_r<5>(L);
    case 6: return launch_r<6>(L);
    case 7: return launch_r<7>(L);
    case 8: return launch_r<8>(L);
    default: return hipErrorNotSupported;
  }
}

// B_dy fragment table for a 2D FP32 operator of radius R <= 8: for every dy
// (d = dy + R) and lane (n = lane % 16, g = lane / 16), the eight bf16 values
// B_dy[8g + j][n] = W[dy][8g + j - n - R] inside the band, else 0; hi plane
// then lo plane (lo = bf16(w - hi)).  Layout: [2d + plane][lane][8] uint16.
std::vector<uint16_t> mfma_b_table(const std::vector<float> &w, int R) {
  const int S = 2 * R + 1;
  std::vector<uint16_t> t((size_t)2 * S * 64 * 8, 0);
  for (int d = 0; d < S; ++d)
    for (int lane = 0; lane < 64; ++lane)
      for (int j = 0; j < 8; ++j) {
        const int n = lane % 16, g = lane / 16;
        const int dx = 8 * g + j - n - R;
        if (dx < -R || dx > R) continue;
        const float x = w[(size_t)d * S + (dx + R)];
        const uint16_t hi = bf16_host(x);
        float hf;
        const uint32_t hb = (uint32_t)hi << 16;
        std::memcpy(&hf, &hb, 4);
        t[(((size_t)(2 * d) * 64) + lane) * 8 + j] = hi;
        t[(((size_t)(2 * d + 1) * 64) + lane) * 8 + j] = bf16_host(x - hf);
      }
  return t;
}

}  // namespace stencil
