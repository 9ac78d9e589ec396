// 2D sweep with K time steps per pass over HBM (temporal blocking in
// registers), bit-identical to K separate plain sweeps.
//
// The paper keeps several steps of a tile on chip with tessellate tiling
// (Section 3.4) so data is not reloaded between steps.  Here a wavefront
// streams a strip of 256 FP32 (128 FP64) columns down y through a pipeline of
// K stages: stage s turns rows of time level s into rows of level s+1 with
// the accumulator queue of the single-step kernel (2R+1 pending rows in
// registers, 16 bytes of columns per lane, the R columns beyond them fetched
// from the neighbouring lanes by DPP) and hands each finished row straight to
// stage s+1.  Only level 0 is read from HBM and only level K is written.
//
// Each level loses R valid columns at both ends of the strip (strips do not
// exchange halos), so a strip loads its span of columns and stores the
// middle span - 2B, B = K*R rounded up to a whole 16-byte vector; rows likewise: a
// strip of BY output rows streams BY + 2KR input rows, and rows of a level
// that lack history only ever feed rows of the next level that are not
// stored.  Every stored value went through K plain steps in the canonical
// order (acc = +0, one FMA per tap, offsets row-major), so the result equals
// K plain sweeps bit for bit.
//
// ZB (Dirichlet boundary): the grid is a padded copy (pad >= R on every
// face) holding the ghost value; each stage sets its output to that value
// outside the interior box, so every level is the Dirichlet sweep's and the
// pad keeps its value.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <utility>

#include "internal.h"
#include "sweep2d_common.h"

namespace stencil {

namespace {

using k2d::fmat;
using k2d::in_mask;
using k2d::load_vec;
using k2d::store_vec;
using k2d::WArr;
using k2d::wrap1;

// A lane holds 16 bytes of a row (4 FP32 or 2 FP64 columns, one vector load
// each, so a wavefront's load covers 1 KiB contiguously): a strip spans 256
// FP32 or 128 FP64 columns.
template <typename T>
__host__ __device__ constexpr int lane_cols() { return 16 / (int)sizeof(T); }
template <typename T>
__host__ __device__ constexpr int span_cols() { return 64 * lane_cols<T>(); }
// Columns a strip discards on each side: K*R rounded up to whole lanes.
template <typename T>
__host__ __device__ constexpr int border(int K, int R) {
  return (K * R + lane_cols<T>() - 1) / lane_cols<T>() * lane_cols<T>();
}

// Blocks are dealt round-robin to the 8 XCDs (block b to XCD b mod 8):
// renumber them so each XCD runs one contiguous range of strips, for any
// block count, and neighbouring strips share halo lines in one L2.
__device__ __forceinline__ int xcd_contiguous(int b, int nb) {
  const int x = b & 7, i = b >> 3, q = nb >> 3, r = nb & 7;
  return x * q + min(x, r) + i;
}

// Whole-wavefront DPP shifts by one lane: lane i receives lane i-1's value
// (shr) or lane i+1's (shl); the end lanes receive 0.
__device__ __forceinline__ float lane_from_left(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x),
                                                                0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_from_right(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x),
                                                                0x130, 0xF, 0xF, true));
}
// FP64: the two 32-bit halves moved by the same shifts
__device__ __forceinline__ double lane_from_left(double x) {
  const int2 h = __builtin_bit_cast(int2, x);
  return __builtin_bit_cast(double, make_int2(
      __builtin_amdgcn_update_dpp(0, h.x, 0x138, 0xF, 0xF, true),
      __builtin_amdgcn_update_dpp(0, h.y, 0x138, 0xF, 0xF, true)));
}
__device__ __forceinline__ double lane_from_right(double x) {
  const int2 h = __builtin_bit_cast(int2, x);
  return __builtin_bit_cast(double, make_int2(
      __builtin_amdgcn_update_dpp(0, h.x, 0x130, 0xF, 0xF, true),
      __builtin_amdgcn_update_dpp(0, h.y, 0x130, 0xF, 0xF, true)));
}

// acc + w * (a neighbouring lane's x), the lane shift done by the FMA's own
// DPP source operand (lanes at the wavefront's end read 0, as above).  The
// compiler folds a DPP move into adds and multiplies but not into an FMA with
// an accumulator, and it cannot see the DPP read inside the asm: the s_nop
// gives the two wait states a DPP read needs after a VALU write of its
// source.  FIRST: the sum starts from +0 (acc is not read).
template <bool LEFT, bool FIRST>
__device__ __forceinline__ float fma_lane(float x, float w, float acc) {
  if constexpr (FIRST) {
    float r;
    if constexpr (LEFT)
      asm("s_nop 1\n\tv_mov_b32 %0, 0\n\tv_fmac_f32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf "
          "bank_mask:0xf bound_ctrl:1" : "=&v"(r) : "v"(x), "v"(w));
    else
      asm("s_nop 1\n\tv_mov_b32 %0, 0\n\tv_fmac_f32_dpp %0, %1, %2 wave_shl:1 row_mask:0xf "
          "bank_mask:0xf bound_ctrl:1" : "=&v"(r) : "v"(x), "v"(w));
    return r;
  } else {
    if constexpr (LEFT)
      asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 wave_shr:1 row_mask:0xf bank_mask:0xf "
          "bound_ctrl:1" : "+v"(acc) : "v"(x), "v"(w));
    else
      asm("s_nop 1\n\tv_fmac_f32_dpp %0, %1, %2 wave_shl:1 row_mask:0xf bank_mask:0xf "
          "bound_ctrl:1" : "+v"(acc) : "v"(x), "v"(w));
    return acc;
  }
}

template <typename F, int... Ks>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Ks...>) {
  (f(std::integral_constant<int, Ks>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Strip layout of a launch: tiles_x strip columns; columns [mx0, mx1) hold
// strips of by rows, the others (zero-boundary launches: the columns whose
// strips hold pad columns, which mask every stage per lane) shorter strips
// of by_m rows, numbered first.
struct TbTiling {
  int tiles_x, by, mx0, mx1, by_m, tiles_y_m;
};

// One strip (column tx, output rows [y0, y1)).  ZB: zero every stage's
// output outside zbox.
template <typename T, int R, int MASK, int K, bool ZB>
__device__ __forceinline__ void tb_body(const T *__restrict__ in, T *__restrict__ out,
                                        int ny, int nx,
                                        const WArr<T, (2 * R + 1) * (2 * R + 1)> &W,
                                        int4 zbox, T zval, int tx, int y0, int y1) {
  constexpr int S = 2 * R + 1;
  constexpr int NU = S;                        // queue length = unroll of the row loop
  constexpr int kVX = lane_cols<T>();
  constexpr int kSpan = span_cols<T>();
  constexpr int B = border<T>(K, R);
  constexpr int WOUT = kSpan - 2 * B;          // stored columns per strip
  static_assert(WOUT > 0, "strip geometry");
  static_assert(R <= kVX, "halo columns come from the two neighbouring lanes");

  const int lane = threadIdx.x;
  const int xo0 = tx * WOUT;     // first stored column of the strip
  const int xi0 = xo0 - B;       // first loaded column (a multiple of kVX)
  const int jstart = y0 - K * R, jend = y1 + K * R;  // level-0 rows streamed
  // The lane's columns xi0 + kVX*lane .. + kVX - 1 wrap as a whole (nx % kVX == 0).
  const int gx = wrap1(xi0 + kVX * lane, nx);
  // Stored lanes: their columns inside [B, kSpan - B) and inside the grid.
  const int lo = kVX * lane - B;
  const bool store_ok = lo >= 0 && lo + kVX <= WOUT && xo0 + lo + kVX <= nx;
  // ZB: the lane's columns inside the interior box (zbox = rows [x, y),
  // columns [z, w)).  Indices are taken unwrapped: a column or row past the
  // pad lies outside the grid too, where every value is 0.
  bool col_in[kVX];
#pragma unroll
  for (int v = 0; v < kVX; ++v)
    col_in[v] = !ZB || (xi0 + kVX * lane + v >= zbox.z && xi0 + kVX * lane + v < zbox.w);
  // most strips hold no pad column: their rows are masked whole (uniform)
  const bool cols_in = !ZB || (xi0 >= zbox.z && xi0 + kSpan <= zbox.w);

  // FP32 radius 1: the lane shifts are done by the FMAs' own DPP source
  // operands (at larger radii the waits they need cost more than the moves
  // they save); the weights of those taps in VGPRs (an operand beside a DPP
  // source must be one)
  constexpr bool kDppFma = sizeof(T) == 4 && R == 1;
  T wv[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) {
    if constexpr (kDppFma) {
      float r;
      asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(W[i]));
      wv[i] = r;
    } else {
      wv[i] = W[i];
    }
  }

  T acc[K][NU][kVX];
#pragma unroll
  for (int s = 0; s < K; ++s)
#pragma unroll
    for (int k = 0; k < NU; ++k)
#pragma unroll
      for (int v = 0; v < kVX; ++v) acc[s][k][v] = T(0);

  // One level-0 row j through the K stages; u = (j - jstart) mod NU.  PRO
  // (the first rows of a strip): stage s runs only from j - jstart = 2sR on.
  auto row = [&](const int j, const int u, const T (&in_row)[kVX], auto na)
                 __attribute__((always_inline)) {
    // NA: stages to run (a compile-time count), or -1: stage s from
    // j - jstart = 2sR on
    constexpr int NA = decltype(na)::value;
    constexpr bool PRO = NA < 0;
    T cur[kVX];
#pragma unroll
    for (int v = 0; v < kVX; ++v) cur[v] = in_row[v];
    // Stage s takes level-s row j - s*R and finishes level-(s+1) row
    // j - (s+1)*R; the slot of an output row is fixed by its index mod NU.
#pragma unroll
    for (int s = 0; s < (NA < 0 ? K : NA); ++s) {
      if (PRO && j - jstart < 2 * s * R) break;  // uniform: later stages start later
      // the R columns on either side come from the neighbouring lanes (FP32
      // radius 1: read by the FMAs themselves)
      T win[kVX + 2 * R];
#pragma unroll
      for (int i = 0; i < R; ++i)
        win[i] = kDppFma ? T(0) : lane_from_left(cur[kVX - R + i]);
#pragma unroll
      for (int v = 0; v < kVX; ++v) win[R + v] = cur[v];
#pragma unroll
      for (int i = 0; i < R; ++i)
        win[R + kVX + i] = kDppFma ? T(0) : lane_from_right(cur[i]);
      // input row j feeds output rows j-R+k with vertical offset oy = R-k;
      // for each output row the offsets arrive with oy ascending, and the
      // first one (k = 2R) starts the sum from +0 in place of a cleared slot
#pragma unroll
      for (int k = S - 1; k >= 0; --k) {
        const int slot = (u + k) % NU;
        const int oy = R - k;
#pragma unroll
        for (int ox = -R; ox <= R; ++ox) {
          if (in_mask<MASK, R>(oy, ox)) {
            const T wt = W[(oy + R) * S + (ox + R)];
            const bool first = k == S - 1 && ox == (MASK == MASK_BOX ? -R : 0);
#pragma unroll
            for (int v = 0; v < kVX; ++v) {
              const int c = v + ox;  // the tap's column, relative to the lane's first
              if constexpr (kDppFma) {
                const T wr = wv[(oy + R) * S + (ox + R)];
                if (c < 0)
                  acc[s][slot][v] = first ? fma_lane<true, true>(cur[kVX + c], wr, T(0))
                                          : fma_lane<true, false>(cur[kVX + c], wr, acc[s][slot][v]);
                else if (c >= kVX)
                  acc[s][slot][v] = first ? fma_lane<false, true>(cur[c - kVX], wr, T(0))
                                          : fma_lane<false, false>(cur[c - kVX], wr, acc[s][slot][v]);
                else
                  acc[s][slot][v] = fmat(wt, cur[c], first ? T(0) : acc[s][slot][v]);
              } else {
                acc[s][slot][v] = fmat(wt, win[R + c], first ? T(0) : acc[s][slot][v]);
              }
            }
          }
        }
      }
#pragma unroll
      for (int v = 0; v < kVX; ++v) cur[v] = acc[s][u % NU][v];
      if constexpr (ZB) {
        // level-(s+1) row j - (s+1)R: zero outside the interior box
        const int yr = j - (s + 1) * R;
        const bool row_in = yr >= zbox.x && yr < zbox.y;
        if (!cols_in || !row_in) {
#pragma unroll
          for (int v = 0; v < kVX; ++v) cur[v] = (row_in && col_in[v]) ? cur[v] : zval;
        }
      }
    }
    // level-K row just completed; a stored row has j - jstart >= 2KR, where
    // every stage runs
    const int yd = j - K * R;
    if (store_ok && yd >= y0 && yd < y1) store_vec<T, kVX>(out + (size_t)yd * nx + xo0 + lo, cur);
  };

  // Level-0 rows arrive a group of NU rows ahead: a group's loads are issued
  // before the previous group's K*NU stage updates, which cover their
  // latency (one row per wavefront in flight does not).  Two buffers
  // alternate, so no register with a load in flight is ever copied (a copy
  // makes the compiler wait for every outstanding access), and the loads are
  // unconditional for the same reason: rows past the end re-read the last.
  auto fetch = [&](const int j0, T (&buf)[NU][kVX]) __attribute__((always_inline)) {
#pragma unroll
    for (int p = 0; p < NU; ++p)
      load_vec<T, kVX>(in + (size_t)wrap1(min(j0 + p, jend - 1), ny) * nx + gx, buf[p]);
  };
  T bufA[NU][kVX], bufB[NU][kVX];
  fetch(jstart, bufA);
  // The first level-s row that a stored row depends on is streamed at index
  // 2sR (index = j - jstart): before it stage s computes nothing that is
  // kept (its earlier outputs lie outside the strip's dependency trapezoid
  // and reach stage s+1 only before that stage starts).  The first PG groups
  // of NU rows run only the stages that matter, which skips R*K*(K-1) of the
  // strip's K*(BY + 2KR) stage-rows.  Every output slot restarts from +0 at
  // its first tap, so a stage that starts late needs no cleared queue.
  constexpr int PG = ((2 * (K - 1) * R + NU - 1) / NU + 1) / 2 * 2;
  // (unrolled for FP32 operators of radius <= 2; for the others the unrolled
  // form raised the registers past an occupancy step or measured slower)
  constexpr bool kStaticPrologue = sizeof(T) == 4 && R <= 2;
  // Pairs of NU-row groups: up to 2NU-1 rows past jend are computed and
  // dropped (the launch sizes strips to avoid them).
  auto pair = [&](const int jb, auto pro) __attribute__((always_inline)) {
    fetch(jb + NU, bufB);
#pragma unroll
    for (int u = 0; u < NU; ++u) row(jb + u, u, bufA[u], pro);
    fetch(jb + 2 * NU, bufA);
#pragma unroll
    for (int u = 0; u < NU; ++u) row(jb + NU + u, u, bufB[u], pro);
  };
  int jb = jstart;
  if constexpr (kStaticPrologue) {
    // unrolled: row i of the prologue runs its min(K, i/(2R) + 1) stages
    static_for<PG / 2>([&](auto pc) __attribute__((always_inline)) {
      constexpr int p0 = 2 * decltype(pc)::value * NU;
      fetch(jb + p0 + NU, bufB);
      static_for<NU>([&](auto uc) __attribute__((always_inline)) {
        constexpr int u = decltype(uc)::value;
        row(jb + p0 + u, u, bufA[u], std::integral_constant<int, std::min(K, (p0 + u) / (2 * R) + 1)>{});
      });
      fetch(jb + p0 + 2 * NU, bufA);
      static_for<NU>([&](auto uc) __attribute__((always_inline)) {
        constexpr int u = decltype(uc)::value;
        row(jb + p0 + NU + u, u, bufB[u],
            std::integral_constant<int, std::min(K, (p0 + NU + u) / (2 * R) + 1)>{});
      });
    });
    jb += PG * NU;
  } else {
    for (; jb < jstart + PG * NU; jb += 2 * NU) pair(jb, std::integral_constant<int, -1>{});
  }
  for (; jb < jend; jb += 2 * NU) pair(jb, std::integral_constant<int, K>{});
}

// All strips of a launch are resident at once (one per wavefront slot), so
// the launch lasts as long as its slowest strip: a zero-boundary launch runs
// the masked body in every strip (an unmasked body for the strips that hold
// no pad cell measured no faster), and the strips that hold pad columns are
// shorter.
template <typename T, int R, int MASK, int K, bool ZB>
__global__ void __launch_bounds__(64)
k_sweep2d_tb(const T *__restrict__ in, T *__restrict__ out, int ny, int nx, TbTiling tl,
             WArr<T, (2 * R + 1) * (2 * R + 1)> W, int4 zbox, T zval) {
  int t = xcd_contiguous(blockIdx.x, gridDim.x);
  const int ncm = tl.mx0 + (tl.tiles_x - tl.mx1);  // strip columns of short strips
  int tx, y0, by;
  if (t < ncm * tl.tiles_y_m) {
    const int c = t / tl.tiles_y_m;
    tx = c < tl.mx0 ? c : tl.mx1 + (c - tl.mx0);
    y0 = (t - c * tl.tiles_y_m) * tl.by_m;
    by = tl.by_m;
  } else {
    t -= ncm * tl.tiles_y_m;
    const int w = tl.mx1 - tl.mx0;
    tx = tl.mx0 + t % w;
    y0 = (t / w) * tl.by;
    by = tl.by;
  }
  tb_body<T, R, MASK, K, ZB>(in, out, ny, nx, W, zbox, zval, tx, y0, min(y0 + by, ny));
}

// Wavefront slots the device holds at once for a kernel (one wave per block).
template <typename F>
int resident_blocks(F kernel) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 256 * 8;
  }
  return std::max(1, cus * per_cu);
}

template <typename T, int R, int MASK, int K>
hipError_t launch_one(const SweepLaunch &L) {
  if (L.zb && (L.zbox[0] < R || L.zbox[2] < R || (int)L.g.ny - L.zbox[1] < R ||
               (int)L.g.nx - L.zbox[3] < R))
    return hipErrorInvalidValue;  // the pad must hold every read of the interior
  constexpr int S = 2 * R + 1;
  constexpr int WOUT = span_cols<T>() - 2 * border<T>(K, R);
  WArr<T, S * S> W;
  for (int i = 0; i < S * S; ++i) W.v[i] = sizeof(T) == 4 ? (T)L.op->w32[i] : (T)L.op->w64[i];
  const int ny = (int)L.g.ny, nx = (int)L.g.nx;
  const int tiles_x = (nx + WOUT - 1) / WOUT;
  static const int env_by = [] {
    const char *e = std::getenv("STENCIL_TB_ROWS");
    return e ? std::atoi(e) : 0;
  }();
  int by = env_by;
  if (by <= 0) {
    // One strip per resident wavefront slot, each as tall as that allows
    // (a second round of strips measured slower than taller strips, whose
    // 2KR redundant rows cost less); at least 4KR rows.
    static const int slots = resident_blocks(k_sweep2d_tb<T, R, MASK, K, false>);
    const int tiles_y = std::max(1, slots / tiles_x);
    by = std::max((ny + tiles_y - 1) / tiles_y, 4 * K * R);
    // whole pairs of (2R+1)-row groups per strip: no rows past its end
    const int pair = 2 * S;
    by += (pair - (by + 2 * K * R) % pair) % pair;
  }
  by = std::min(by, ny);
  TbTiling tl{tiles_x, by, 0, tiles_x, by, 1};
  if (L.zb) {
    // strip columns whose strips hold pad columns: a prefix and a suffix
    constexpr int SPAN = span_cols<T>(), B = border<T>(K, R);
    auto masked = [&](int tx) { return tx * WOUT - B < L.zbox[2] || tx * WOUT - B + SPAN > L.zbox[3]; };
    int mx0 = 0, mx1 = tiles_x;
    while (mx0 < tiles_x && masked(mx0)) ++mx0;
    while (mx1 > mx0 && masked(mx1 - 1)) --mx1;
    if (mx0 > 0 || mx1 < tiles_x) {
      // their per-lane masking makes a row dearer: 70% of the others' height
      // (8192^2 star, 12 steps: 3894 GStencil/s at 100%, 4029 at 85%, 4140
      // at 75% and at 65%); STENCIL_TB_EDGE_PCT sets another percentage
      static const int pct = [] {
        const char *e = std::getenv("STENCIL_TB_EDGE_PCT");
        return e ? std::max(10, std::min(100, std::atoi(e))) : 70;
      }();
      const int pair = 2 * S;
      int by_m = std::max(by * pct / 100, 4 * K * R);
      by_m += (pair - (by_m + 2 * K * R) % pair) % pair;
      tl = TbTiling{tiles_x, by, mx0, mx1, std::min(by_m, ny), 1};
      tl.tiles_y_m = (ny + tl.by_m - 1) / tl.by_m;
    }
  }
  const int ncm = tl.mx0 + (tiles_x - tl.mx1);
  const int64_t blocks = (int64_t)ncm * tl.tiles_y_m + (int64_t)(tl.mx1 - tl.mx0) * ((ny + by - 1) / by);
  if (blocks > (1LL << 31) - 1) return hipErrorNotSupported;
  const int4 zbox = {L.zbox[0], L.zbox[1], L.zbox[2], L.zbox[3]};
  if (L.zb)
    hipLaunchKernelGGL((k_sweep2d_tb<T, R, MASK, K, true>), dim3((unsigned)blocks), dim3(64), 0,
                       L.stream, (const T *)L.in, (T *)L.out, ny, nx, tl, W, zbox, (T)L.zval);
  else
    hipLaunchKernelGGL((k_sweep2d_tb<T, R, MASK, K, false>), dim3((unsigned)blocks), dim3(64), 0,
                       L.stream, (const T *)L.in, (T *)L.out, ny, nx, tl, W, zbox, T(0));
  return hipGetLastError();
}

// The launch of L.steps (2 .. KMAX) fused applications.
template <typename T, int R, int MASK, int... Ks>
hipError_t launch_ks(const SweepLaunch &L, std::integer_sequence<int, Ks...>) {
  hipError_t e = hipErrorNotSupported;
  ((L.steps == Ks + 2 ? (void)(e = launch_one<T, R, MASK, Ks + 2>(L)) : (void)0), ...);
  return e;
}
template <typename T, int R, int MASK, int KMAX>
hipError_t launch_upto(const SweepLaunch &L) {
  return launch_ks<T, R, MASK>(L, std::make_integer_sequence<int, KMAX - 1>{});
}

// Most steps per pass by radius: the queue (K*(2R+1) rows of 16 bytes per
// lane) and two groups of 2R+1 prefetched rows must leave room for two or
// more waves/SIMD.  Boxes of radius 3 and more
// (49+ taps per point) are bound by FMA issue in one step per pass already,
// and fusing only adds the redundant border work.
int tb_max(int R, int mask, int dtype) {
  if (mask == MASK_BOX && R >= 3) return 1;
  static const int star1 = [] {
    const char *e = std::getenv("STENCIL_TB_STAR_K");
    return e ? std::max(2, std::min(14, std::atoi(e))) : 0;
  }();
  if (dtype == STENCIL_F64) {
    // the FP64 star: 14 steps (8192^2: 2939 GStencil/s against 2832 at 12,
    // 2880 at 13; 15 and 16 exceed the registers of two wavefronts per SIMD:
    // 2664, 2658)
    if (R == 1) return mask == MASK_BOX ? 8 : (star1 ? star1 : 14);
    return R == 2 ? 4 : 1;
  }
  // FP32 radius-1 star: 10 steps, where the kernel (149 VGPRs) holds three
  // wavefronts per SIMD; 12 need 186 and allow two (8192^2 on one GPU: 5155
  // GStencil/s at 10 against 5064 at 12, the zero-boundary star 4488 against
  // 4222; 11 capped to three wavefronts spills, 12 capped spills more)
  if (R == 1 && mask != MASK_BOX) return star1 ? std::min(star1, 12) : 10;
  return R == 1 ? 8 : R == 2 ? 4 : R <= 4 ? 2 : 1;
}

template <typename T>
hipError_t launch_t(const SweepLaunch &L) {
  const bool box = L.op->mask == MASK_BOX;  // the diamond contains the axes
  if constexpr (sizeof(T) == 4) {
    switch (L.op->R) {
      case 1: return box ? launch_upto<T, 1, MASK_BOX, 8>(L) : launch_upto<T, 1, MASK_DIAMOND, 12>(L);
      case 2: return box ? launch_upto<T, 2, MASK_BOX, 4>(L) : launch_upto<T, 2, MASK_DIAMOND, 4>(L);
      case 3: return box ? hipErrorNotSupported : launch_upto<T, 3, MASK_DIAMOND, 2>(L);
      case 4: return box ? hipErrorNotSupported : launch_upto<T, 4, MASK_DIAMOND, 2>(L);
      default: return hipErrorNotSupported;
    }
  } else {
    switch (L.op->R) {
      case 1: return box ? launch_upto<T, 1, MASK_BOX, 8>(L) : launch_upto<T, 1, MASK_DIAMOND, 14>(L);
      case 2: return box ? launch_upto<T, 2, MASK_BOX, 4>(L) : launch_upto<T, 2, MASK_DIAMOND, 4>(L);
      default: return hipErrorNotSupported;
    }
  }
}

}  // namespace

int sweep2d_max_steps(const SweepLaunch &L) {
  const int R = L.op->R;
  const int K = tb_max(R, L.op->mask, L.dtype);
  if (K < 2 || L.g.dim != 2) return 1;
  const int vx = L.dtype == STENCIL_F64 ? lane_cols<double>() : lane_cols<float>();
  if (L.g.nx % vx != 0 || L.g.nx < 64 * vx || L.g.ny < 2 * K * R + 1) return 1;
  if (L.g.nx > (1 << 30) || L.g.ny > (1 << 30)) return 1;
  return K;
}

hipError_t launch_sweep2d_tb(const SweepLaunch &L) {
  if (L.steps < 2 || L.steps > sweep2d_max_steps(L)) return hipErrorNotSupported;
  if ((uintptr_t)L.in % 16 != 0 || (uintptr_t)L.out % 16 != 0) return hipErrorNotSupported;
  return L.dtype == STENCIL_F32 ? launch_t<float>(L) : launch_t<double>(L);
}

}  // namespace stencil
