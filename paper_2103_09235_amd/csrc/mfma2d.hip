// Folded 2D stencil as banded-Toeplitz matrix products on the gfx950 matrix
// cores (v_mfma_f32_16x16x32_bf16), with BF16 hi+lo splitting of both
// operands and FP32 accumulation.
//
// Folding m steps (Section 3.3) turns a 3x3 box into a dense (2R+1)^2 box,
// R = m*r, dense enough that one output row is a sum of matrix products.
// For one input row j and one vertical offset dy, the contribution to the
// output row y = j - dy, for 16 blocks of 16 consecutive columns, is
//   D[n][i] = sum_k T_dy[n][k] * U_j[k][i],
//   T_dy[n][k] = W[dy][k - n - R] if |k-n-R| <= R  (16 x 32, banded Toeplitz),
//   U_j[k][i]  = u[j][16 i - R + k]              (32 x 16: block i's window),
// with D[n][i] the output at column 16 i + n of the strip and K = 32 >=
// 16 + 2R for R <= 8.  So each input row is converted to matrix operands
// once and feeds the 2R+1 output rows it touches (the rows pending in a
// register queue, as in the vector sweeps): three products per (row, dy),
// hi*hi, lo*hi and hi*lo of bf16 hi = bf16(x) and lo = bf16(x - hi), all into
// one FP32 accumulator per pending output row.  The split recovers about 16
// significant bits, so the result stays within 1e-3 of the FP64 sweep over
// hundreds of folded steps, unlike a single BF16 product.  The matrix unit
// adds in its own order, so this form does not keep the canonical summation
// order.
//
// Work layout: one wavefront per strip of 256 output columns and a segment
// of rows, streaming down the rows.  Lane l (i = l % 16, g = l / 16) holds
// U_j[8g .. 8g+7][i], 8 consecutive input values it loads straight from
// memory, and the accumulator values D[4g .. 4g+3][i], 4 consecutive output
// columns it stores with one 16-byte store.  Every input row has a register
// buffer of its own among 2R+1: the loads of row t+2R+1 are issued while row
// t is multiplied.  The T_dy fragments (hi and lo) stay in registers for the
// whole kernel, loaded from a table the host builds once per operator.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <utility>

#include "internal.h"

namespace stencil {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

constexpr int kStrip = 256;  // output columns per wavefront (16 blocks of 16)

__device__ __forceinline__ int wrapfull(int i, int n) {
  const int r = i % n;
  return r < 0 ? r + n : r;
}

// Blocks are dealt round-robin to the 8 XCDs (block b to XCD b mod 8):
// renumber them so that each XCD runs one contiguous range of strips and
// neighbouring strips share their halo columns in one L2.
__device__ __forceinline__ int xcd_contiguous(int b, int nb) {
  const int x = b & 7, i = b >> 3, q = nb >> 3, r = nb & 7;
  return x * q + min(x, r) + i;
}

// Calls f(std::integral_constant<int, K>) for K = 0 .. N-1 in order.
template <typename F, int... Ks>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Ks...>) {
  (f(std::integral_constant<int, Ks>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// V: floats per load (4: the window starts are multiples of 4, rows hold a
// multiple of 4 floats and the input is 16-byte aligned, so a vector never
// straddles the periodic seam; 2 likewise; 1: any shape).  FULL: every
// strip of the launch holds 256 columns of the grid (x0 + 256 <= nx, nx a
// multiple of 4, output 16-byte aligned); otherwise the strips start at
// x_first and are stored column by column.
template <int R, int V, bool FULL>
__global__ void __launch_bounds__(64)
k_mfma2d(const float *__restrict__ in, float *__restrict__ out, int ny, int nx, int rows,
         int tiles_x, int x_first, const uint4 *__restrict__ btab) {
  static_assert(R >= 1 && R <= 8, "K = 32 covers 16 + 2R columns for R <= 8");
  static_assert(V == 1 || V == 2 || V == 4, "vector width");
  constexpr int S = 2 * R + 1;
  constexpr int NP = 8 / V;  // loads per row and lane
  const int lane = threadIdx.x;
  const int tile = xcd_contiguous(blockIdx.x, gridDim.x);
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int x0 = x_first + tx * kStrip, y0 = ty * rows;
  const int nt = min(rows, ny - y0) + 2 * R;  // input rows streamed

  // T_dy fragments: lane (n = lane % 16, g = lane / 16) holds k = 8g .. 8g+7;
  // btab[(2d) * 64 + lane] = hi, btab[(2d + 1) * 64 + lane] = lo, d = dy + R
  bf16x8 th[S], tl[S];
#pragma unroll
  for (int d = 0; d < S; ++d) {
    th[d] = __builtin_bit_cast(bf16x8, btab[(2 * d) * 64 + lane]);
    tl[d] = __builtin_bit_cast(bf16x8, btab[(2 * d + 1) * 64 + lane]);
  }

  const int i = lane & 15, g = lane >> 4;
  const int c0 = x0 + 16 * i - R + 8 * g;  // first input column of the lane's window
  int col[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) col[p] = wrapfull(c0 + V * p, nx);

  float buf[S][8];
  auto load = [&](float(&b)[8], int gy) {
    const float *src = in + (size_t)gy * nx;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if constexpr (V == 4) {
        const f32x4 v = *reinterpret_cast<const f32x4 *>(src + col[p]);
        b[4 * p] = v[0]; b[4 * p + 1] = v[1]; b[4 * p + 2] = v[2]; b[4 * p + 3] = v[3];
      } else if constexpr (V == 2) {
        const f32x2 v = *reinterpret_cast<const f32x2 *>(src + col[p]);
        b[2 * p] = v[0]; b[2 * p + 1] = v[1];
      } else {
        b[p] = src[col[p]];
      }
    }
  };
  // rows stream from y0 - R; the loads run S rows ahead of the products
  // (rows past the segment wrap around the grid: always in bounds)
  int gy = wrapfull(y0 - R, ny);
#pragma unroll
  for (int u = 0; u < S; ++u) {
    load(buf[u], gy);
    gy = gy + 1 == ny ? 0 : gy + 1;
  }
  f32x4 acc[S];
#pragma unroll
  for (int d = 0; d < S; ++d) acc[d] = f32x4{0.f, 0.f, 0.f, 0.f};
  const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
  const int oc = x0 + 16 * i + 4 * g;  // first output column of the lane
  float *orow = out + (size_t)y0 * nx + oc;  // output row of step t = 2R

  // hi = bf16(x), lo = bf16(x - hi), both rounded to nearest even by the
  // packed conversion; hi is widened back by a shift or a mask of its pair
  auto split = [](const float(&x)[8], bf16x8 &h, bf16x8 &l) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bf16x2 p = __builtin_convertvector(f32x2{x[2 * q], x[2 * q + 1]}, bf16x2);
      const unsigned pu = __builtin_bit_cast(unsigned, p);
      const float h0 = __builtin_bit_cast(float, pu << 16);
      const float h1 = __builtin_bit_cast(float, pu & 0xFFFF0000u);
      const bf16x2 lp = __builtin_convertvector(f32x2{x[2 * q] - h0, x[2 * q + 1] - h1}, bf16x2);
      h[2 * q] = p[0];
      h[2 * q + 1] = p[1];
      l[2 * q] = lp[0];
      l[2 * q + 1] = lp[1];
    }
  };

  // Step t (U = t mod S): input row y0 - R + t from buffer U; the output row
  // y = y0 + t - R - dy accumulates in slot (t - R - dy) mod S = (U - d) mod
  // S (d = dy + R), so slot U starts a new row (d = 0) and slot (U + 1) mod
  // S completes one (d = 2R), stored at the end of the step from t = 2R on.
  // LOAD: refill buffer U with the row S steps ahead.  (Converting the next
  // row during this step's products, to overlap the two, needs registers
  // this form does not have: it measured slower.)
  auto step = [&](auto uc, int t, auto load_c, auto store_c) {
    constexpr int U = decltype(uc)::value;
    constexpr bool LOAD = decltype(load_c)::value, STORE = decltype(store_c)::value;
    bf16x8 ah, al;
    split(buf[U], ah, al);
    if constexpr (LOAD) {
      load(buf[U], gy);
      gy = gy + 1 == ny ? 0 : gy + 1;
    }
    // the completing slot first, so its products are done by the store
    constexpr int SC = (U + 1) % S;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const bf16x8 a = p == 1 ? al : ah;
      acc[SC] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(p == 2 ? tl[2 * R] : th[2 * R], a,
                                                        acc[SC], 0, 0, 0);
#pragma unroll
      for (int d = 0; d < 2 * R; ++d) {
        const int sl = ((U - d) % S + S) % S;
        acc[sl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            p == 2 ? tl[d] : th[d], a, (p == 0 && d == 0) ? zero : acc[sl], 0, 0, 0);
      }
    }
    if constexpr (STORE) {
      float *dst = orow + (size_t)(t - 2 * R) * nx;
      if constexpr (FULL) {
        __builtin_nontemporal_store(acc[SC], reinterpret_cast<f32x4 *>(dst));
      } else {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj)
          if (oc + jj < nx) __builtin_nontemporal_store(acc[SC][jj], dst + jj);
      }
    }
  };
  using yes = std::true_type;
  using no = std::false_type;
  // the first 2R steps complete no output row
  static_for<2 * R>([&](auto k) { step(k, (int)decltype(k)::value, yes{}, no{}); });
  // whole rounds of S steps: one straight-line body without branches, so
  // every step's loads are issued where they stand
  int t0 = 2 * R;
  for (; t0 + S <= nt; t0 += S)
    static_for<S>([&](auto k) {
      constexpr int K = decltype(k)::value;
      step(std::integral_constant<int, (2 * R + K) % S>{}, t0 + K, yes{}, yes{});
    });
  // the last steps (fewer than S) consume buffers already loaded
  static_for<S - 1>([&](auto k) {
    constexpr int K = decltype(k)::value;
    if (t0 + K < nt)
      step(std::integral_constant<int, (2 * R + K) % S>{}, t0 + K, no{}, yes{});
  });
}

// Wavefront slots the device holds at once for a kernel (one wave per block).
template <typename F>
int resident_waves(F kernel) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 256 * 4;
  }
  return std::max(1, cus * per_cu);
}

template <int R, int V, bool FULL>
hipError_t launch_rvf(const SweepLaunch &L, int tiles_x, int x_first) {
  constexpr int S = 2 * R + 1;
  const int ny = (int)L.g.ny;
  static const int env_rows = [] {
    const char *e = std::getenv("STENCIL_MFMA_ROWS");
    return e ? std::atoi(e) : 0;
  }();
  int rows = env_rows;
  if (rows <= 0) {
    // one strip per resident wavefront slot, each as tall as that allows
    static const int slots = resident_waves(k_mfma2d<R, V, true>);
    const int tiles_y = std::max(1, slots / tiles_x);
    rows = (ny + tiles_y - 1) / tiles_y;
  }
  rows = std::min(std::max(rows, 2 * S), ny);
  const int tiles_y = (ny + rows - 1) / rows;
  const int64_t blocks = (int64_t)tiles_x * tiles_y;
  if (blocks > (1LL << 31) - 1) return hipErrorNotSupported;
  hipLaunchKernelGGL((k_mfma2d<R, V, FULL>), dim3((unsigned)blocks), dim3(64), 0, L.stream,
                     (const float *)L.in, (float *)L.out, ny, (int)L.g.nx, rows, tiles_x,
                     x_first, (const uint4 *)L.op->mfma_b);
  return hipGetLastError();
}

// Whole 256-column strips in one launch, the remaining columns (a grid
// narrower than a strip, or every column when output rows are not whole
// 16-byte vectors) in a second launch that stores column by column.
template <int R, int V>
hipError_t launch_rv(const SweepLaunch &L) {
  const int nx = (int)L.g.nx;
  const bool vec_out = nx % 4 == 0 && (uintptr_t)L.out % 16 == 0;
  const int full = vec_out ? nx / kStrip : 0;
  if (full > 0) {
    hipError_t e = launch_rvf<R, V, true>(L, full, 0);
    if (e != hipSuccess) return e;
  }
  const int rest = nx - full * kStrip;
  if (rest > 0) return launch_rvf<R, V, false>(L, (rest + kStrip - 1) / kStrip, full * kStrip);
  return hipSuccess;
}

template <int R>
hipError_t launch_r(const SweepLaunch &L) {
  if (!L.op->mfma_b) return hipErrorNotSupported;
  const int64_t nx = L.g.nx;
  const uintptr_t a = (uintptr_t)L.in;
  if constexpr (R % 4 == 0)
    if (nx % 4 == 0 && a % 16 == 0) return launch_rv<R, 4>(L);
  if constexpr (R % 2 == 0)
    if (nx % 2 == 0 && a % 8 == 0) return launch_rv<R, 2>(L);
  return launch_rv<R, 1>(L);
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
