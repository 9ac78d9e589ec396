// Batched sweeps: many independent 2D grids of uneven sizes and mixed
// stencils advanced together.
//
// Small grids waste a GPU when launched one by one (a 64 x 64 grid is 16 KB
// of traffic, far below a launch's fixed cost).  Here every (folded) sweep
// of every grid is one persistent launch: the host cuts all grids into tiles
// (one wavefront streams one tile, as in the single-grid 2D sweep), sorts
// them by decreasing cost, and each workgroup takes tiles round-robin,
// branching per tile (never per lane) to the kernel variant of that grid's
// operator.  Grids of at least 256 columns instead run their
// (folded) applications several per launch in fused strips, before the
// one-step launches of the rest.  All launches of the time loop, plus one
// copy for grids whose launch count is odd, are captured once in a hipGraph
// and replayed.  The fold depth m of each grid is chosen per (stencil, size
// class) by timing the candidates on the device (the paper leaves parameter
// tuning to future work, evaluation section) and cached on disk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <list>
#include <map>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "internal.h"
#include "sweep2d_impl.h"

namespace stencil {

namespace {

constexpr int kMaxBatchRadius = 2;  // operators the batched kernel carries
constexpr int kTileRows = 64;

struct GridInfo {
  float *data;
  float *scratch;
  int nx, ny;
  int q, s;          // folded sweeps first, then plain sweeps
  int var_f, var_p;  // kernel variant of the folded and the plain operator
  int w_f, w_p;      // offsets of their weights in the weight table
  // Grids that a strip layout fits fuse the folded (or, at m = 1, the
  // plain) applications: fpass passes of the fused kernel first, the
  // applications spread evenly (the first nfull passes run tail + 1, the
  // others tail); the one-step launches then run the plain remainder only.
  int fpass, nfull, tail;
  int bord;  // columns a fused strip discards on each side (>= the pass's K*R)
};

struct Tile {
  int grid, x0, y0, y1;
};

// variant = (R - 1) * 4 + (mask == DIAMOND) * 2 + (vector lanes)
__host__ __device__ constexpr int variant_id(int R, bool diamond, bool vx4) {
  return (R - 1) * 4 + (diamond ? 2 : 0) + (vx4 ? 1 : 0);
}
__host__ __device__ constexpr bool variant_diamond(int var) { return (var & 2) != 0; }

// applications of a fused grid's pass k (k < fpass)
__host__ __device__ inline int pass_apps(const GridInfo &g, int k) {
  return k < g.nfull ? g.tail + 1 : g.tail;
}

// Variants: aligned rows of >= 256 floats use vector lanes (two rows of
// look-ahead), the rest strided lanes (4 coalesced scalars per lane).
__global__ void __launch_bounds__(64)
k_batched(const Tile *__restrict__ tiles, int ntiles, const GridInfo *__restrict__ grids,
          const float *__restrict__ wtab, int k) {
  using k2d::sweep2d_tile;
  using k2d::WPtr;
  __shared__ float lds[2 * k2d::lds_row<kMaxBatchRadius, 4>(0)];  // largest variant
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const Tile tl = tiles[t];
    const GridInfo g = grids[tl.grid];
    // fused grids: only the plain remainder (s sweeps) after fpass passes
    const int q = g.fpass ? 0 : g.q;
    if (k >= q + g.s) continue;
    const bool folded = k < q;
    const int var = folded ? g.var_f : g.var_p;
    const WPtr<float> w{wtab + (folded ? g.w_f : g.w_p)};
    const int par = (k + g.fpass) & 1;
    const float *in = par ? g.scratch : g.data;
    float *out = par ? g.data : g.scratch;
    switch (var) {
      case variant_id(1, false, false):
        sweep2d_tile<float, 1, MASK_BOX, 4, 1, true, false>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, w, lds);
        break;
      case variant_id(1, false, true):
        sweep2d_tile<float, 1, MASK_BOX, 4, 2, false, false>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, w, lds);
        break;
      case variant_id(1, true, false):
        sweep2d_tile<float, 1, MASK_DIAMOND, 4, 1, true, false>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, w, lds);
        break;
      case variant_id(1, true, true):
        sweep2d_tile<float, 1, MASK_DIAMOND, 4, 2, false, false>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, w, lds);
        break;
      case variant_id(2, false, false):
        sweep2d_tile<float, 2, MASK_BOX, 4, 1, true, false>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, w, lds);
        break;
      case variant_id(2, false, true):
        sweep2d_tile<float, 2, MASK_BOX, 4, 2, false, false>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, w, lds);
        break;
      case variant_id(2, true, false):
        sweep2d_tile<float, 2, MASK_DIAMOND, 4, 1, true, false>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, w, lds);
        break;
      default:
        sweep2d_tile<float, 2, MASK_DIAMOND, 4, 2, false, false>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, w, lds);
        break;
    }
  }
}

// ------------------------------------------------------------ fused passes
//
// The fused 2D strip (several applications of one operator per pass, one
// wavefront per 256-column strip streaming down y, each application a
// pipeline stage with its own accumulator queue, neighbour columns by DPP;
// the single-grid form is described with the fused 2D sweep) with KC <= KMAX
// applications, a compile-time count: each pass launches the kernel of every
// KC its grids take in that pass (blocks of other grids return at once), so
// a short pass costs its own stages only (a runtime count would make the
// compiler drain every outstanding load where stage branches merge).
// A grid's strips keep the border of its largest pass (its fused-step cap,
// at most KMAX), so one tiling serves every KC it uses.  Canonical order,
// bit-identical to KC single applications.

// Strip height (rows a fused strip stores): the default, or the
// STENCIL_BATCH_TB_ROWS override, which also fixes it for the tuner.
static int tb_rows_env() {
  static const int rows = [] {
    const char *e = std::getenv("STENCIL_BATCH_TB_ROWS");
    return e ? std::max(16, std::atoi(e)) : 0;
  }();
  return rows;
}
static int tb_rows() { return tb_rows_env() ? tb_rows_env() : 64; }

__device__ __forceinline__ float tb_from_left(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x),
                                                                0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float tb_from_right(float x) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, x),
                                                                0x130, 0xF, 0xF, true));
}

__host__ __device__ constexpr int tb_border(int K, int R) { return (K * R + 3) / 4 * 4; }
__host__ __device__ constexpr int tb_kmax(int R) { return R == 1 ? 8 : 4; }

// VX columns per lane (4, 2 or 1: strips of 256, 128 or 64 columns; the
// narrow ones cover a grid's last columns, or a whole narrow grid, with less
// discarded border work); VX >= R, so a neighbour column is at most one lane
// away.  VEC (VX = 4 only): rows of whole 16-byte vectors (one vector load
// and store per lane and row); otherwise VX scalar loads, each column wrapped
// on its own, and stores column by column.  The strip's columns must span
// less than twice the grid's width (each column wraps at most once):
// 64 * VX - B - 2 < nx.
template <int R, int MASK, int VX, bool VEC, int K>
__device__ void tb_strip(const float *__restrict__ in, float *__restrict__ out, int ny, int nx,
                         int xo0, int y0, int y1, const float *__restrict__ wt, const int B) {
  static_assert(VX >= R && (!VEC || VX == 4), "strip layout");
  using k2d::fmat;
  using k2d::in_mask;
  using k2d::load_vec;
  using k2d::store_vec;
  using k2d::wrap1;
  constexpr int S = 2 * R + 1;
  constexpr int NU = S;
  constexpr int KMAX = tb_kmax(R);
  static_assert(K >= 1 && K <= KMAX, "stages per pass");
  const int WOUT = 64 * VX - 2 * B;  // B >= K * R: the host's strip plan
  float W[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) W[i] = wt[i];
  const int lane = threadIdx.x;
  const int gx = wrap1(xo0 - B + VX * lane, nx);
  int gxs[VX];  // scalar path: each column wrapped on its own
#pragma unroll
  for (int v = 0; v < VX; ++v) gxs[v] = wrap1(xo0 - B + VX * lane + v, nx);
  const int lo = VX * lane - B;
  const bool store_ok = lo >= 0 && lo + VX <= WOUT && xo0 + lo + VX <= nx;
  bool store_v[VX];
#pragma unroll
  for (int v = 0; v < VX; ++v) store_v[v] = lo + v >= 0 && lo + v < WOUT && xo0 + lo + v < nx;
  const int jstart = y0 - K * R, jend = y1 + K * R;
  float acc[K][NU][VX];
#pragma unroll
  for (int st = 0; st < K; ++st)
#pragma unroll
    for (int k = 0; k < NU; ++k)
#pragma unroll
      for (int v = 0; v < VX; ++v) acc[st][k][v] = 0.0f;
  // One level-0 row j through the stages; u = (j - jstart) mod NU.  NA: the
  // number of stages (a compile-time count), or -1: stage st from
  // j - jstart = 2 st R on.
  auto row = [&](const int j, const int u, const float (&in_row)[VX], auto na)
                 __attribute__((always_inline)) {
    constexpr int NA = decltype(na)::value;
    float cur[VX];
#pragma unroll
    for (int v = 0; v < VX; ++v) cur[v] = in_row[v];
#pragma unroll
    for (int st = 0; st < (NA < 0 ? K : NA); ++st) {
      if (NA < 0 && j - jstart < 2 * st * R) break;  // uniform: later stages start later
      {
        float win[VX + 2 * R];
#pragma unroll
        for (int i = 0; i < R; ++i) win[i] = tb_from_left(cur[VX - R + i]);
#pragma unroll
        for (int v = 0; v < VX; ++v) win[R + v] = cur[v];
#pragma unroll
        for (int i = 0; i < R; ++i) win[R + VX + i] = tb_from_right(cur[i]);
#pragma unroll
        for (int k = S - 1; k >= 0; --k) {
          const int slot = (u + k) % NU;
          const int oy = R - k;
#pragma unroll
          for (int ox = -R; ox <= R; ++ox) {
            if (in_mask<MASK, R>(oy, ox)) {
              const float w = W[(oy + R) * S + (ox + R)];
              const bool first = k == S - 1 && ox == (MASK == MASK_BOX ? -R : 0);
#pragma unroll
              for (int v = 0; v < VX; ++v)
                acc[st][slot][v] = fmat(w, win[R + v + ox], first ? 0.0f : acc[st][slot][v]);
            }
          }
        }
#pragma unroll
        for (int v = 0; v < VX; ++v) cur[v] = acc[st][u % NU][v];
      }
    }
    const int yd = j - K * R;
    if (yd >= y0 && yd < y1) {
      float *dst = out + (size_t)yd * nx + xo0 + lo;
      const float(&val)[VX] = cur;
      if constexpr (VEC) {
        if (store_ok) store_vec<float, 4>(dst, val);
      } else {
#pragma unroll
        for (int v = 0; v < VX; ++v)
          if (store_v[v]) dst[v] = val[v];
      }
    }
  };
  auto fetch = [&](const int j0, float (&buf)[NU][VX]) __attribute__((always_inline)) {
#pragma unroll
    for (int p = 0; p < NU; ++p) {
      const float *rowp = in + (size_t)wrap1(min(j0 + p, jend - 1), ny) * nx;
      if constexpr (VEC) {
        load_vec<float, 4>(rowp + gx, buf[p]);
      } else {
#pragma unroll
        for (int v = 0; v < VX; ++v) buf[p][v] = rowp[gxs[v]];
      }
    }
  };
  float bufA[NU][VX], bufB[NU][VX];
  fetch(jstart, bufA);
  // Stage st computes nothing that a stored row depends on before streamed
  // row 2 st R (as in the single-grid fused kernel): the first PG groups of
  // NU rows run only the stages that matter (R*K*(K-1) of a strip's
  // K*(BY + 2KR) stage-rows skipped).  Rows past jend are skipped too (a
  // uniform branch per row; their loads stay unconditional).
  constexpr int PG = ((2 * (K - 1) * R + NU - 1) / NU + 1) / 2 * 2;
  auto pair = [&](const int jb, auto na) __attribute__((always_inline)) {
    fetch(jb + NU, bufB);
#pragma unroll
    for (int u = 0; u < NU; ++u)
      if (jb + u < jend) row(jb + u, u, bufA[u], na);
    fetch(jb + 2 * NU, bufA);
#pragma unroll
    for (int u = 0; u < NU; ++u)
      if (jb + NU + u < jend) row(jb + NU + u, u, bufB[u], na);
  };
  int jb = jstart;
  for (; jb < jstart + PG * NU; jb += 2 * NU) pair(jb, std::integral_constant<int, -1>{});
  for (; jb < jend; jb += 2 * NU) pair(jb, std::integral_constant<int, K>{});
}

// Pass k of every fused grid whose pass k has KC applications: one block per
// strip.  One kernel per radius, row layout and KC, so that each gets its own
// register allocation (a kernel holding every variant would run all of them
// at the occupancy of the largest).
template <int R, int VX, bool VEC, int KC>
__global__ void __launch_bounds__(64)
k_batched_tb(const Tile *__restrict__ tiles, const GridInfo *__restrict__ grids,
             const float *__restrict__ wtab, int k) {
  // each XCD (blocks are dealt to the 8 XCDs round-robin) takes one
  // contiguous range of strips, so neighbouring strips share their
  // overlapping rows and columns in one L2
  const int bi = blockIdx.x, nb = gridDim.x;
  const int x = bi & 7, q = nb >> 3, r = nb & 7;
  const Tile tl = tiles[x * q + min(x, r) + (bi >> 3)];
  const GridInfo g = grids[tl.grid];
  if (k >= g.fpass || pass_apps(g, k) != KC) return;
  const float *in = (k & 1) ? g.scratch : g.data;
  float *out = (k & 1) ? g.data : g.scratch;
  const float *w = wtab + g.w_f;
  if (variant_diamond(g.var_f))
    tb_strip<R, MASK_DIAMOND, VX, VEC, KC>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, w, g.bord);
  else
    tb_strip<R, MASK_BOX, VX, VEC, KC>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, w, g.bord);
}

// Strip layouts of the fused passes, and their tile groups: group =
// (R - 1) * kTbLayouts + layout (radius 2 has no one-column layout).
enum TbLayout { kTb4 = 0, kTb4Vec = 1, kTb2 = 2, kTb1 = 3, kTbLayouts = 4 };
constexpr int kTbGroups = 2 * kTbLayouts;
__host__ __device__ constexpr int tb_vx(int layout) {
  return layout == kTb2 ? 2 : layout == kTb1 ? 1 : 4;
}
// output columns of a strip: 64 * VX lanes' columns minus the border B each side
__host__ __device__ constexpr int tb_wout(int B, int layout) {
  return 64 * tb_vx(layout) - 2 * B;
}
// the strip's columns wrap at most once: 64 * VX - B - 2 < nx
__host__ __device__ constexpr int tb_min_nx(int B, int layout) {
  return 64 * tb_vx(layout) - B - 1;
}

// Grids whose total sweep count is odd end in scratch: copy them back.
__global__ void __launch_bounds__(256)
k_batched_copyback(const GridInfo *__restrict__ grids, const int *__restrict__ odd, int nodd) {
  using V = __attribute__((ext_vector_type(4))) float;
  for (int i = blockIdx.y; i < nodd; i += gridDim.y) {
    const GridInfo g = grids[odd[i]];
    const int64_t n = (int64_t)g.nx * g.ny;
    const int64_t stride = (int64_t)gridDim.x * 256;
    int64_t head = 0;  // 16-byte vectors where both buffers allow them
    if ((((uintptr_t)g.data | (uintptr_t)g.scratch) & 15) == 0) {
      head = n / 4 * 4;
      const V *src = reinterpret_cast<const V *>(g.scratch);
      V *dst = reinterpret_cast<V *>(g.data);
      for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < n / 4; e += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + e), dst + e);
    }
    for (int64_t e = head + blockIdx.x * 256 + threadIdx.x; e < n; e += stride)
      g.data[e] = g.scratch[e];
  }
}

// Column strips (layout, first column) of a fused grid with border B:
// 256-column strips while whole ones fit, then the cheapest cover of the
// remaining columns: one more wide strip, or 128-column strips followed by
// 64-column ones, priced by their lanes' columns times a per-layout cost per
// column (the narrow layouts spend relatively more on neighbour exchange and
// loop work).  narrow: no 256-column strips where the narrow layouts can
// cover the grid (more, shorter-lived wavefronts per row band).  Empty when
// no layout fits the grid's width (then it is not fused).
std::vector<std::pair<int, int>> strip_plan(int nx, int R, bool vec, int B, bool narrow) {
  constexpr double kCost[kTbLayouts] = {1.0, 1.0, 1.15, 1.4};
  std::vector<std::pair<int, int>> out;
  const bool ok2 = nx >= tb_min_nx(B, kTb2);
  const bool ok1 = R == 1 && nx >= tb_min_nx(B, kTb1);
  const bool ok4 = nx >= tb_min_nx(B, kTb4) && !(narrow && (ok2 || ok1));
  const int w4 = tb_wout(B, kTb4), w2 = tb_wout(B, kTb2), w1 = tb_wout(B, kTb1);
  const int wide = vec ? kTb4Vec : kTb4;
  int x = 0;
  if (ok4)
    for (; nx - x >= w4; x += w4) out.push_back({wide, x});
  const int rem = nx - x;
  if (rem == 0) return out;
  double best = ok4 ? 256 * kCost[kTb4] : 1e30;
  int ba = -1, bb = 0;
  const int amax = ok2 ? (rem + w2 - 1) / w2 : 0;
  for (int a = 0; a <= amax; ++a) {
    const int left = std::max(0, rem - a * w2);
    if (left > 0 && !ok1) continue;
    const int b = left > 0 ? (left + w1 - 1) / w1 : 0;
    const double c = a * 128 * kCost[kTb2] + b * 64 * kCost[kTb1];
    if (c < best) {
      best = c;
      ba = a;
      bb = b;
    }
  }
  if (ba < 0) {
    if (!ok4) return {};
    out.push_back({wide, x});
    return out;
  }
  for (int a = 0; a < ba; ++a, x += w2) out.push_back({kTb2, x});
  for (int b = 0; b < bb; ++b, x += w1) out.push_back({kTb1, x});
  return out;
}

// --------------------------------------------------------------- tuning

int size_class(int64_t side) {
  int b = 0;
  while ((int64_t)1 << (b + 1) <= side) ++b;
  return b;  // floor(log2(side))
}

struct TuneKey {
  int shape, r, cls;
  bool operator<(const TuneKey &o) const {
    return std::tie(shape, r, cls) < std::tie(o.shape, o.r, o.cls);
  }
};

// A class's tuned choice: fold depth, fused-strip height (0 = default), cap
// on the applications of one fused pass (0 = the kernel's KMAX; a lower cap
// narrows the strips' discarded border) and the strip layout (narrow: 128-
// and 64-column strips only).
struct TuneVal {
  int m = 1, rows = 0, kc = 0, narrow = 0;
  bool operator==(const TuneVal &o) const {
    return m == o.m && rows == o.rows && kc == o.kc && narrow == o.narrow;
  }
};

std::mutex g_mu;
std::map<std::string, std::map<TuneKey, TuneVal>> g_tune;  // per cache file ("" = memory only)

// Cache file lines: "stencil-batched-m shape r cls m" and, optionally,
// "stencil-batched-rows shape r cls rows", "stencil-batched-kc shape r cls
// kc", "stencil-batched-narrow shape r cls 0|1".
void load_tune_file(const std::string &path, std::map<TuneKey, TuneVal> &out) {
  if (path.empty()) return;
  std::ifstream f(path);
  std::string tag;
  int shape, r, cls, v;
  while (f >> tag >> shape >> r >> cls >> v) {
    if (tag == "stencil-batched-m") out[TuneKey{shape, r, cls}].m = v;
    if (tag == "stencil-batched-rows") out[TuneKey{shape, r, cls}].rows = std::max(0, v);
    if (tag == "stencil-batched-kc") out[TuneKey{shape, r, cls}].kc = std::max(0, v);
    if (tag == "stencil-batched-narrow") out[TuneKey{shape, r, cls}].narrow = v ? 1 : 0;
  }
}

void save_tune_file(const std::string &path, const std::map<TuneKey, TuneVal> &tab) {
  if (path.empty()) return;
  std::ofstream f(path, std::ios::trunc);
  for (const auto &kv : tab) {
    const TuneKey &k = kv.first;
    const TuneVal &v = kv.second;
    const std::string id = std::to_string(k.shape) + " " + std::to_string(k.r) + " " +
                           std::to_string(k.cls) + " ";
    f << "stencil-batched-m " << id << v.m << "\n";
    if (v.rows) f << "stencil-batched-rows " << id << v.rows << "\n";
    if (v.kc) f << "stencil-batched-kc " << id << v.kc << "\n";
    if (v.narrow) f << "stencil-batched-narrow " << id << v.narrow << "\n";
  }
}

// Folded FP32 weights of a plan at depth m (cached in the plan).
int plan_weights32(stencil_plan p, int m, const std::vector<float> *&out) {
  auto it = p->batch_w32.find(m);
  if (it == p->batch_w32.end()) {
    std::vector<double> Wm;
    int rc = fold_on_device(p->w, p->dim, p->r, m, Wm);
    if (rc) return rc;
    std::vector<float> W32;
    round_fold_f32(p->w, Wm, p->dim, m * p->r, m, W32);
    it = p->batch_w32.emplace(m, std::move(W32)).first;
  }
  out = &it->second;
  return STENCIL_OK;
}

// ---------------------------------------------------------- batch cache

struct BatchEntry {
  std::vector<uint64_t> key;  // signature: run settings, then 6 words per grid
  int device = 0;
  Tile *d_tiles_tb = nullptr;  // fused strips (one block each), by group
  int tb_off[kTbGroups + 1] = {};
  std::vector<std::tuple<int, int, int>> tb_launch;  // (pass, group, applications)
  Tile *d_tiles = nullptr;
  GridInfo *d_grids = nullptr;
  float *d_w = nullptr;
  int *d_odd = nullptr;
  int ntiles = 0, nodd = 0, launches = 0, nblocks = 0;
  std::vector<int> passes;  // per grid: launches that read and write it
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t graph_stream = nullptr;
};

std::list<BatchEntry> g_cache;  // most recent first
constexpr size_t kCacheEntries = 4;

void free_entry(BatchEntry &b) {
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(b.device);
  (void)hipDeviceSynchronize();
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  if (b.graph) (void)hipGraphDestroy(b.graph);
  if (b.d_tiles) (void)hipFree(b.d_tiles);
  if (b.d_tiles_tb) (void)hipFree(b.d_tiles_tb);
  if (b.d_grids) (void)hipFree(b.d_grids);
  if (b.d_w) (void)hipFree(b.d_w);
  if (b.d_odd) (void)hipFree(b.d_odd);
  (void)hipSetDevice(cur);
}

// The fused-pass kernel of a tile group for KC applications per pass.
template <int R, int VX, bool VEC, int... Ks>
const void *tb_kernel_kc(int kc, std::integer_sequence<int, Ks...>) {
  const void *f = nullptr;
  ((kc == Ks + 1 ? (f = reinterpret_cast<const void *>(&k_batched_tb<R, VX, VEC, Ks + 1>)) : f), ...);
  return f;
}
const void *tb_kernel(int grp, int kc) {
  using K1 = std::make_integer_sequence<int, tb_kmax(1)>;
  using K2 = std::make_integer_sequence<int, tb_kmax(2)>;
  switch (grp) {
    case kTb4: return tb_kernel_kc<1, 4, false>(kc, K1());
    case kTb4Vec: return tb_kernel_kc<1, 4, true>(kc, K1());
    case kTb2: return tb_kernel_kc<1, 2, false>(kc, K1());
    case kTb1: return tb_kernel_kc<1, 1, false>(kc, K1());
    case kTbLayouts + kTb4: return tb_kernel_kc<2, 4, false>(kc, K2());
    case kTbLayouts + kTb4Vec: return tb_kernel_kc<2, 4, true>(kc, K2());
    case kTbLayouts + kTb2: return tb_kernel_kc<2, 2, false>(kc, K2());
    default: return nullptr;  // no one-column strips at radius 2
  }
}

hipError_t enqueue(const BatchEntry &b, hipStream_t s) {
  for (const auto &l : b.tb_launch) {
    int k = std::get<0>(l);
    const int grp = std::get<1>(l), kc = std::get<2>(l);
    const int n = b.tb_off[grp + 1] - b.tb_off[grp];
    const void *f = tb_kernel(grp, kc);
    if (n == 0 || !f) return hipErrorInvalidValue;
    const Tile *t = b.d_tiles_tb + b.tb_off[grp];
    const GridInfo *g = b.d_grids;
    const float *w = b.d_w;
    void *args[] = {&t, &g, &w, &k};
    hipError_t e = hipLaunchKernel(f, dim3(n), dim3(64), args, 0, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  for (int k = 0; k < b.launches; ++k) {
    hipLaunchKernelGGL(k_batched, dim3(b.nblocks), dim3(64), 0, s, b.d_tiles, b.ntiles,
                       b.d_grids, b.d_w, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (b.nodd > 0) {
    // enough blocks per grid that a few large grids still fill the chip
    const int by = std::min(b.nodd, 4096), bx = std::max(64, 4096 / by);
    hipLaunchKernelGGL(k_batched_copyback, dim3(bx, by), dim3(256), 0, s,
                       b.d_grids, b.d_odd, b.nodd);
    return hipGetLastError();
  }
  return hipSuccess;
}

// Builds a batch: fold weights, fused strips and one-step tiles per grid,
// device tables, and (use_graph) the captured time loop.
int build_entry(const stencil_plan *plans, const stencil_grid *grids, int count, int64_t T,
                const std::vector<TuneVal> &cfg, bool use_graph, int device, BatchEntry &b) {
  b.device = device;
  std::vector<GridInfo> gi(count);
  std::vector<float> wt;
  std::map<std::pair<stencil_plan, int>, int> woff;
  auto weights_at = [&](stencil_plan p, int m, int *off) -> int {
    auto f = woff.find({p, m});
    if (f != woff.end()) {
      *off = f->second;
      return STENCIL_OK;
    }
    const std::vector<float> *w;
    int rc = plan_weights32(p, m, w);
    if (rc) return rc;
    *off = (int)wt.size();
    wt.insert(wt.end(), w->begin(), w->end());
    woff[{p, m}] = *off;
    return STENCIL_OK;
  };
  std::vector<std::pair<int64_t, Tile>> tiles, tiles_tb[kTbGroups];
  std::set<std::tuple<int, int, int>> tb_need;  // (pass, group, applications)
  std::vector<int> odd;
  int launches = 0;
  for (int i = 0; i < count; ++i) {
    const stencil_plan p = plans[i];
    const stencil_grid &g = grids[i];
    const int m = cfg[i].m;
    GridInfo &G = gi[i];
    G.data = (float *)g.data;
    G.scratch = (float *)g.scratch;
    G.ny = (int)g.shape[0];
    G.nx = (int)g.shape[1];
    G.q = m > 1 ? (int)(T / m) : 0;
    G.s = m > 1 ? (int)(T % m) : (int)T;
    const bool vx4 = (G.nx % 4 == 0) && ((uintptr_t)g.data % 16 == 0) &&
                     ((uintptr_t)g.scratch % 16 == 0);
    const bool star = p->shape == STENCIL_STAR;
    G.var_p = variant_id(p->r, star, vx4);
    G.var_f = variant_id(m * p->r, star, vx4);
    int rc = weights_at(p, 1, &G.w_p);
    if (rc) return rc;
    G.w_f = G.w_p;
    if (m > 1 && (rc = weights_at(p, m, &G.w_f))) return rc;
    const int R = m * p->r;
    // fused passes: the folded applications (the plain ones at m = 1) of
    // grids that some strip layout fits, up to KM (the class's cap, at most
    // tb_kmax(R)) per pass; the strips discard a border of KM * R columns
    G.fpass = G.nfull = G.tail = 0;
    const int KM = R <= kMaxBatchRadius
                       ? (cfg[i].kc > 0 ? std::min(cfg[i].kc, tb_kmax(R)) : tb_kmax(R)) : 1;
    G.bord = tb_border(KM, R);
    const std::vector<std::pair<int, int>> strips =
        R <= kMaxBatchRadius && G.ny >= 2 * KM * R + 1
            ? strip_plan(G.nx, R, vx4, G.bord, cfg[i].narrow != 0)
            : std::vector<std::pair<int, int>>();
    if (!strips.empty()) {
      const int apps = m > 1 ? G.q : G.s;
      const int rest = m > 1 ? G.s : 0;
      if (apps > 1) {
        // the fewest passes, applications spread evenly (pass k takes
        // tail + 1 while k < nfull, else tail).  An odd launch count is not
        // made even by one more pass: a pass costs more than copying the
        // grid back
        G.fpass = (apps + KM - 1) / KM;
        G.tail = apps / G.fpass;
        G.nfull = apps % G.fpass;
        G.q = 0;
        G.s = rest;
      }
    }
    const int sweeps = G.fpass + (G.fpass ? G.s : G.q + G.s);
    b.passes.push_back(sweeps);
    launches = std::max(launches, G.fpass ? G.s : G.q + G.s);
    if (sweeps % 2) odd.push_back(i);
    if (G.fpass) {
      const int kk = pass_apps(G, 0);
      const int rows = cfg[i].rows > 0 ? cfg[i].rows : tb_rows();
      for (int y0 = 0; y0 < G.ny; y0 += rows)
        for (const auto &st : strips) {
          const int y1 = std::min(G.ny, y0 + rows);
          const int64_t cost = (int64_t)(y1 - y0 + 2 * kk * R) * kk * (2 * R + 1) * tb_vx(st.first);
          tiles_tb[(R - 1) * kTbLayouts + st.first].push_back({cost, Tile{i, st.second, y0, y1}});
        }
      // the kernels pass k launches: (group, applications) of this grid
      for (const auto &st : strips)
        for (int k = 0; k < G.fpass; ++k)
          tb_need.insert({k, (R - 1) * kTbLayouts + st.first, pass_apps(G, k)});
    }
    const int bx = 256;
    const int Rp = G.fpass ? p->r : R;  // one-step work of fused grids is plain
    if (G.fpass == 0 || G.s > 0)
      for (int y0 = 0; y0 < G.ny; y0 += kTileRows)
        for (int x0 = 0; x0 < G.nx; x0 += bx) {
          const int y1 = std::min(G.ny, y0 + kTileRows);
          const int64_t cost = (int64_t)(y1 - y0 + 2 * Rp) * (2 * Rp + 1);
          tiles.push_back({cost, Tile{i, x0, y0, y1}});
        }
  }
  auto by_cost = [](const auto &a, const auto &b) { return a.first > b.first; };
  std::stable_sort(tiles.begin(), tiles.end(), by_cost);
  std::vector<Tile> tl(tiles.size()), tltb;
  for (size_t t = 0; t < tiles.size(); ++t) tl[t] = tiles[t].second;
  for (int grp = 0; grp < kTbGroups; ++grp) {
    // strips in grid, row band, column order (neighbours adjacent); every
    // block is resident at once or nearly, so cost order matters little
    static const bool by_cost_env = std::getenv("STENCIL_BATCH_TB_SORT") != nullptr;
    if (by_cost_env) std::stable_sort(tiles_tb[grp].begin(), tiles_tb[grp].end(), by_cost);
    b.tb_off[grp] = (int)tltb.size();
    for (const auto &ct : tiles_tb[grp]) tltb.push_back(ct.second);
  }
  b.tb_off[kTbGroups] = (int)tltb.size();
  if (tltb.size() > (size_t)((1LL << 31) - 1)) return fail(STENCIL_E_UNSUPPORTED, "batch too large");
  b.ntiles = (int)tl.size();
  b.nodd = (int)odd.size();
  b.launches = b.ntiles ? launches : 0;
  b.tb_launch.assign(tb_need.begin(), tb_need.end());
  hipDeviceProp_t prop;
  STENCIL_HIP_TRY(hipGetDeviceProperties(&prop, device));
  b.nblocks = std::max(1, std::min(b.ntiles, prop.multiProcessorCount * 32));
  hipError_t e = hipMalloc(&b.d_tiles, sizeof(Tile) * std::max<size_t>(1, tl.size()));
  if (e == hipSuccess) e = hipMalloc(&b.d_tiles_tb, sizeof(Tile) * std::max<size_t>(1, tltb.size()));
  if (e == hipSuccess && !tltb.empty())
    e = hipMemcpy(b.d_tiles_tb, tltb.data(), sizeof(Tile) * tltb.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMalloc(&b.d_grids, sizeof(GridInfo) * gi.size());
  if (e == hipSuccess) e = hipMalloc(&b.d_w, sizeof(float) * std::max<size_t>(1, wt.size()));
  if (e == hipSuccess) e = hipMalloc(&b.d_odd, sizeof(int) * std::max<size_t>(1, odd.size()));
  if (e == hipSuccess && !tl.empty())
    e = hipMemcpy(b.d_tiles, tl.data(), sizeof(Tile) * tl.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b.d_grids, gi.data(), sizeof(GridInfo) * gi.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !wt.empty()) e = hipMemcpy(b.d_w, wt.data(), sizeof(float) * wt.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !odd.empty()) e = hipMemcpy(b.d_odd, odd.data(), sizeof(int) * odd.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && use_graph) {
    // capture on a private stream, replayed later on the caller's stream
    e = hipStreamCreateWithFlags(&b.graph_stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(b.graph_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e2 = enqueue(b, b.graph_stream);
      e = hipStreamEndCapture(b.graph_stream, &b.graph);
      if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0);
    if (b.graph_stream) (void)hipStreamDestroy(b.graph_stream);
    b.graph_stream = nullptr;
  }
  if (e != hipSuccess) {
    free_entry(b);
    return hip_fail(e, "batched setup");
  }
  return STENCIL_OK;
}

// The tuner (the paper leaves parameter tuning to future work, evaluation
// section): every (stencil, radius, size class) of the batch that the cache
// does not hold gets a fold depth, a fused-strip height, a cap on the
// applications of a fused pass and a strip layout, chosen by timing the
// whole batch as it runs (same grids, same plans, every class sharing the
// launches with the others) on scratch copies of its buffers: a choice that
// wins for a class alone can lose on the batch by splitting its launches,
// so only the batch's time decides.  Coordinate descent: from the default
// (m = 1, 64 rows, the kernel's cap, widest strips), the classes by
// decreasing share of the batch's points, one parameter at a time over its
// candidates, a change kept only if the batch runs at least 1% faster (ties
// keep the earlier choice: smaller m, default height and cap, wide strips).
// Each timing is the fastest of three runs of min(T, 64) original steps.
int tune_batch(const stencil_plan *plans, const stencil_grid *grids, int count, int64_t T,
               int max_m, hipStream_t stream, int device, std::map<TuneKey, TuneVal> &tab,
               const std::set<TuneKey> &todo) {
  // scratch copies: every grid's two buffers, 256-byte aligned slices
  std::vector<size_t> off(count);
  size_t total = 0;
  for (int i = 0; i < count; ++i) {
    off[i] = total;
    total += ((size_t)grids[i].shape[0] * grids[i].shape[1] * sizeof(float) + 255) / 256 * 256;
  }
  char *pool = nullptr;
  STENCIL_HIP_TRY(hipMalloc(&pool, 2 * total));
  std::vector<stencil_grid> gs(grids, grids + count);
  for (int i = 0; i < count; ++i) {
    gs[i].data = pool + off[i];
    gs[i].scratch = pool + total + off[i];
    gs[i].stream = stream;
  }
  hipError_t he = hipMemsetAsync(pool, 0, 2 * total, stream);
  const int64_t Tt = std::min<int64_t>(T, 64);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (he == hipSuccess) he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  std::vector<TuneKey> key_of(count);
  std::map<TuneKey, double> share;
  for (int i = 0; i < count; ++i) {
    const stencil_plan p = plans[i];
    key_of[i] = TuneKey{p->shape, p->r, size_class(std::min(grids[i].shape[0], grids[i].shape[1]))};
    share[key_of[i]] += (double)grids[i].shape[0] * grids[i].shape[1];
  }
  std::map<TuneKey, TuneVal> cur = tab;
  for (const TuneKey &k : todo) cur[k] = TuneVal();
  int rc = STENCIL_OK;
  // the batch's time with the choices in `c` (ms), or a negative value for a
  // configuration the grids do not admit
  auto time_with = [&](const std::map<TuneKey, TuneVal> &c, double *ms_out) -> int {
    std::vector<TuneVal> cfg(count);
    for (int i = 0; i < count; ++i) {
      cfg[i] = c.at(key_of[i]);
      const int64_t side = std::min(grids[i].shape[0], grids[i].shape[1]);
      const int r = plans[i]->r;
      if (cfg[i].m * r > kMaxBatchRadius || 2 * cfg[i].m * r + 1 > side) {
        *ms_out = -1.0;
        return STENCIL_OK;
      }
    }
    BatchEntry be;
    int rc2 = build_entry(plans, gs.data(), count, Tt, cfg, false, device, be);
    if (rc2) return rc2;
    float best = 1e30f;
    hipError_t e = enqueue(be, stream);  // warm
    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
      e = hipEventRecord(e0, stream);
      if (e == hipSuccess) e = enqueue(be, stream);
      if (e == hipSuccess) e = hipEventRecord(e1, stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float t = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
      best = std::min(best, t);
    }
    free_entry(be);
    if (e != hipSuccess) return hip_fail(e, "batched tuning run");
    *ms_out = best;
    return STENCIL_OK;
  };
  double best_ms = 0.0;
  if (he != hipSuccess) rc = hip_fail(he, "batched tuning setup");
  if (rc == STENCIL_OK) rc = time_with(cur, &best_ms);
  std::vector<TuneKey> order(todo.begin(), todo.end());
  std::stable_sort(order.begin(), order.end(),
                   [&](const TuneKey &a, const TuneKey &b) { return share[a] > share[b]; });
  for (const TuneKey &k : order) {
    if (rc != STENCIL_OK || best_ms <= 0.0) break;
    const int kmax = tb_kmax(std::min(k.r, kMaxBatchRadius));
    for (int param = 0; param < 4 && rc == STENCIL_OK; ++param) {
      std::vector<int> cands;
      if (param == 0)
        for (int m = 1; m <= max_m && m * k.r <= kMaxBatchRadius; ++m) cands.push_back(m);
      if (param == 1) cands = {0, kmax / 2};
      if (param == 2) cands = {0, 32, 128, 256};
      if (param == 3) cands = {0, 1};
      for (int v : cands) {
        std::map<TuneKey, TuneVal> trial = cur;
        TuneVal &tv = trial[k];
        int *field = param == 0 ? &tv.m : param == 1 ? &tv.kc : param == 2 ? &tv.rows : &tv.narrow;
        if (*field == v) continue;
        *field = v;
        double ms = 0.0;
        rc = time_with(trial, &ms);
        if (rc != STENCIL_OK) break;
        if (ms > 0.0 && ms < best_ms * 0.99) {
          best_ms = ms;
          cur = trial;
        }
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(stream);
  (void)hipFree(pool);
  if (rc == STENCIL_OK)
    for (const TuneKey &k : todo) tab[k] = cur[k];
  return rc;
}

}  // namespace

void evict_batched_plan(const stencil_plan_s *p) {
  std::lock_guard<std::mutex> lock(g_mu);
  for (auto it = g_cache.begin(); it != g_cache.end();) {
    bool names = false;
    // words 4 + 6 i hold the plans' ids
    for (size_t k = 4; k < it->key.size() && !names; k += 6) names = it->key[k] == p->id;
    if (names) {
      free_entry(*it);
      it = g_cache.erase(it);
    } else {
      ++it;
    }
  }
}

}  // namespace stencil

using namespace stencil;

extern "C" int stencil_run_batched(const stencil_plan *plans, stencil_grid *grids, int count,
                                   int64_t T, const stencil_batch_opts *opts) {
  set_error("");
  if (count < 0 || T < 0) return fail(STENCIL_E_ARG, "count and T must be >= 0");
  if (count == 0 || T == 0) return STENCIL_OK;
  if (!plans || !grids) return fail(STENCIL_E_ARG, "plans and grids must be non-NULL");
  if (T > (1 << 20)) return fail(STENCIL_E_UNSUPPORTED, "T too large for a batched run");
  const hipStream_t stream = (hipStream_t)grids[0].stream;
  for (int i = 0; i < count; ++i) {
    const stencil_plan p = plans[i];
    const stencil_grid &g = grids[i];
    if (!p || !g.data || !g.scratch) return fail(STENCIL_E_ARG, "NULL plan, data or scratch");
    if (p->dim != 2 || g.dim != 2) return fail(STENCIL_E_UNSUPPORTED, "batched runs are 2D");
    if (p->boundary != STENCIL_PERIODIC)
      return fail(STENCIL_E_UNSUPPORTED, "batched runs are periodic");
    if (g.dtype != STENCIL_F32) return fail(STENCIL_E_UNSUPPORTED, "batched runs are FP32");
    if (p->r > kMaxBatchRadius) return fail(STENCIL_E_UNSUPPORTED, "batched stencils need r <= 2");
    if (g.stream != grids[0].stream) return fail(STENCIL_E_ARG, "all grids must name one stream");
    if (g.shape[0] < 2 * p->r + 1 || g.shape[1] < 2 * p->r + 1 || g.shape[0] > (1 << 20) ||
        g.shape[1] > (1 << 20))
      return fail(STENCIL_E_UNSUPPORTED, "grid sides must be in [2r+1, 2^20]");
    const size_t bytes = (size_t)g.shape[0] * g.shape[1] * 4;
    const char *a = (const char *)g.data, *b = (const char *)g.scratch;
    if (a < b + bytes && b < a + bytes) return fail(STENCIL_E_ARG, "data and scratch overlap");
  }
  const int max_m = opts ? std::max(1, opts->max_m) : 1;
  const bool autotune = opts && opts->autotune;
  const bool use_graph = opts && opts->use_graph;
  std::string cache_path;
  if (opts && opts->tune_cache) cache_path = opts->tune_cache;
  else if (const char *e = std::getenv("STENCIL_TUNE_CACHE")) cache_path = e;

  int device = 0;
  STENCIL_HIP_TRY(hipGetDevice(&device));
  std::lock_guard<std::mutex> lock(g_mu);

  // --- fold depth, strip height, pass cap and strip layout per grid: tuned
  // per (shape, r, size class) on the whole batch, cached
  std::map<TuneKey, TuneVal> &tab = g_tune[cache_path];
  if (tab.empty()) load_tune_file(cache_path, tab);
  std::set<TuneKey> todo;
  for (int i = 0; i < count; ++i) {
    const stencil_plan p = plans[i];
    const TuneKey key{p->shape, p->r, size_class(std::min(grids[i].shape[0], grids[i].shape[1]))};
    if (!tab.count(key)) todo.insert(key);
  }
  if (autotune && !todo.empty()) {
    if (int rc = tune_batch(plans, grids, count, T, max_m, stream, device, tab, todo)) return rc;
    save_tune_file(cache_path, tab);
  }
  std::vector<TuneVal> cfg(count);
  for (int i = 0; i < count; ++i) {
    const stencil_plan p = plans[i];
    const int64_t side = std::min(grids[i].shape[0], grids[i].shape[1]);
    const TuneKey key{p->shape, p->r, size_class(side)};
    auto it = tab.find(key);
    TuneVal v = it != tab.end() ? it->second : TuneVal();
    int m = std::max(1, std::min(v.m, max_m));
    while (m > 1 && (m * p->r > kMaxBatchRadius || 2 * m * p->r + 1 > side)) --m;
    v.m = m;
    v.rows = tb_rows_env() ? 0 : std::max(0, std::min(v.rows, 1 << 16));
    v.kc = std::max(0, std::min(v.kc, 64));
    cfg[i] = v;
  }
  if (opts && opts->chosen_m)
    for (int i = 0; i < count; ++i) opts->chosen_m[i] = cfg[i].m;

  // --- signature of this batch (pointers, sizes, plans, fold depths, T)
  std::vector<uint64_t> key;
  key.reserve(4 + 6 * (size_t)count);
  key.push_back((uint64_t)device);
  key.push_back((uint64_t)T);
  key.push_back(use_graph ? 1 : 0);
  key.push_back((uint64_t)(uintptr_t)stream);
  for (int i = 0; i < count; ++i) {
    key.push_back(plans[i]->id);  // never reused, unlike the plan's address
    key.push_back((uint64_t)(uintptr_t)grids[i].data);
    key.push_back((uint64_t)(uintptr_t)grids[i].scratch);
    key.push_back((uint64_t)grids[i].shape[0]);
    key.push_back((uint64_t)grids[i].shape[1]);
    // the grid's choices: fold depth | pass cap << 8 | narrow << 16 | height << 32
    key.push_back((uint64_t)cfg[i].m | ((uint64_t)cfg[i].kc << 8) |
                  ((uint64_t)cfg[i].narrow << 16) | ((uint64_t)cfg[i].rows << 32));
  }
  auto hit = std::find_if(g_cache.begin(), g_cache.end(),
                          [&](const BatchEntry &b) { return b.key == key; });
  if (hit == g_cache.end()) {
    BatchEntry b;
    b.key = key;
    if (int rc = build_entry(plans, grids, count, T, cfg, use_graph, device, b))
      return rc;
    g_cache.push_front(b);
    if (g_cache.size() > kCacheEntries) {
      free_entry(g_cache.back());
      g_cache.pop_back();
    }
    hit = g_cache.begin();
  } else {
    g_cache.splice(g_cache.begin(), g_cache, hit);
    hit = g_cache.begin();
  }
  hipError_t e = hit->exec ? hipGraphLaunch(hit->exec, stream) : enqueue(*hit, stream);
  if (e != hipSuccess) return hip_fail(e, "batched launch");
  if (opts && opts->passes)
    for (int i = 0; i < count; ++i) opts->passes[i] = hit->passes[i];
  return STENCIL_OK;
}
