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
#include <sstream>
#include <string>
#include <tuple>
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
  // Grids of at least 256 columns fuse the folded (or, at
  // m = 1, the plain) applications: fpass launches of the fused kernel
  // first, nfull of KMAX applications and then one of the remaining tail
  // (< KMAX); the one-step launches then run the plain remainder only.
  int fpass, nfull, tail;
};

struct Tile {
  int grid, x0, y0, y1;
};

// variant = (R - 1) * 4 + (mask == DIAMOND) * 2 + (vector lanes)
__host__ __device__ constexpr int variant_id(int R, bool diamond, bool vx4) {
  return (R - 1) * 4 + (diamond ? 2 : 0) + (vx4 ? 1 : 0);
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
// the single-grid form is described with the fused 2D sweep) with the number
// of applications K <= KMAX.  Full passes compile K = KMAX.  A grid's
// last, shorter pass runs all KMAX stages as well and stores stage K-1's
// output, picked by a select: a branch per stage would make the compiler
// drain every outstanding load where the branches merge, and a body per K
// makes the kernel about twice as large, which measured 10% slower on a
// mixed batch.  Strips keep the KMAX border, so one tiling serves every K.  Canonical order, bit-identical to K single
// applications.

static int tb_rows() {
  static const int rows = [] {
    const char *e = std::getenv("STENCIL_BATCH_TB_ROWS");
    return e ? std::max(16, std::atoi(e)) : 64;
  }();
  return rows;
}

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

// VEC: rows of whole 16-byte vectors (one vector load and store per lane and
// row); otherwise four scalar loads, each column wrapped on its own, and
// stores column by column.
template <int R, int MASK, bool VEC, bool FULL>
__device__ void tb_strip(const float *__restrict__ in, float *__restrict__ out, int ny, int nx,
                         int xo0, int y0, int y1, int Kr, const float *__restrict__ wt) {
  using k2d::fmat;
  using k2d::in_mask;
  using k2d::load_vec;
  using k2d::store_vec;
  using k2d::wrap1;
  constexpr int S = 2 * R + 1;
  constexpr int NU = S;
  constexpr int KMAX = tb_kmax(R);
  constexpr int B = tb_border(KMAX, R);
  constexpr int WOUT = 256 - 2 * B;
  const int K = FULL ? KMAX : Kr;
  float W[S * S];
#pragma unroll
  for (int i = 0; i < S * S; ++i) W[i] = wt[i];
  const int lane = threadIdx.x;
  const int gx = wrap1(xo0 - B + 4 * lane, nx);
  int gxs[4];  // scalar path: each column wrapped on its own
#pragma unroll
  for (int v = 0; v < 4; ++v) gxs[v] = wrap1(xo0 - B + 4 * lane + v, nx);
  const int lo = 4 * lane - B;
  const bool store_ok = lo >= 0 && lo + 4 <= WOUT && xo0 + lo + 4 <= nx;
  bool store_v[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) store_v[v] = lo + v >= 0 && lo + v < WOUT && xo0 + lo + v < nx;
  const int jstart = y0 - K * R, jend = y1 + K * R;
  float acc[KMAX][NU][4];
#pragma unroll
  for (int st = 0; st < KMAX; ++st)
#pragma unroll
    for (int k = 0; k < NU; ++k)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[st][k][v] = 0.0f;
  auto row = [&](const int j, const int u, const float (&in_row)[4]) {
    float cur[4], res[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) cur[v] = res[v] = in_row[v];
#pragma unroll
    for (int st = 0; st < KMAX; ++st) {
      {
        float win[4 + 2 * R];
#pragma unroll
        for (int i = 0; i < R; ++i) win[i] = tb_from_left(cur[4 - R + i]);
#pragma unroll
        for (int v = 0; v < 4; ++v) win[R + v] = cur[v];
#pragma unroll
        for (int i = 0; i < R; ++i) win[R + 4 + i] = tb_from_right(cur[i]);
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
              for (int v = 0; v < 4; ++v)
                acc[st][slot][v] = fmat(w, win[R + v + ox], first ? 0.0f : acc[st][slot][v]);
            }
          }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) cur[v] = acc[st][u % NU][v];
        if constexpr (!FULL) {
#pragma unroll
          for (int v = 0; v < 4; ++v) res[v] = st == K - 1 ? cur[v] : res[v];
        }
      }
    }
    const int yd = j - K * R;
    if (yd >= y0 && yd < y1) {
      float *dst = out + (size_t)yd * nx + xo0 + lo;
      const float(&val)[4] = FULL ? cur : res;
      if constexpr (VEC) {
        if (store_ok) store_vec<float, 4>(dst, val);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (store_v[v]) dst[v] = val[v];
      }
    }
  };
  auto fetch = [&](const int j0, float (&buf)[NU][4]) {
#pragma unroll
    for (int p = 0; p < NU; ++p) {
      const float *rowp = in + (size_t)wrap1(min(j0 + p, jend - 1), ny) * nx;
      if constexpr (VEC) {
        load_vec<float, 4>(rowp + gx, buf[p]);
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) buf[p][v] = rowp[gxs[v]];
      }
    }
  };
  float bufA[NU][4], bufB[NU][4];
  fetch(jstart, bufA);
  for (int jb = jstart; jb < jend; jb += 2 * NU) {
    fetch(jb + NU, bufB);
#pragma unroll
    for (int u = 0; u < NU; ++u) row(jb + u, u, bufA[u]);
    fetch(jb + 2 * NU, bufA);
#pragma unroll
    for (int u = 0; u < NU; ++u) row(jb + NU + u, u, bufB[u]);
  }
}

// One fused pass of every fused grid that has pass k: one block per strip.
// One kernel per radius and row layout, so that each gets its own register
// allocation (a kernel holding every variant would run all of them at the
// occupancy of the largest).
template <int R, bool VEC>
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
  if (k >= g.fpass) return;
  constexpr int KMAX = tb_kmax(R);
  const int K = k < g.nfull ? KMAX : g.tail;
  const float *in = (k & 1) ? g.scratch : g.data;
  float *out = (k & 1) ? g.data : g.scratch;
  const float *w = wtab + g.w_f;
  const bool dia = g.var_f == variant_id(R, true, VEC);
  if (K == KMAX) {
    if (dia) tb_strip<R, MASK_DIAMOND, VEC, true>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, K, w);
    else tb_strip<R, MASK_BOX, VEC, true>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, K, w);
  } else {
    if (dia) tb_strip<R, MASK_DIAMOND, VEC, false>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, K, w);
    else tb_strip<R, MASK_BOX, VEC, false>(in, out, g.ny, g.nx, tl.x0, tl.y0, tl.y1, K, w);
  }
}

// tile groups of the fused passes: (R - 1) * 2 + VEC
constexpr int kTbGroups = 4;

// Grids whose total sweep count is odd end in scratch: copy them back.
__global__ void __launch_bounds__(256)
k_batched_copyback(const GridInfo *__restrict__ grids, const int *__restrict__ odd, int nodd) {
  for (int i = blockIdx.y; i < nodd; i += gridDim.y) {
    const GridInfo g = grids[odd[i]];
    const int64_t n = (int64_t)g.nx * g.ny;
    for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256)
      g.data[e] = g.scratch[e];
  }
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

std::mutex g_mu;
std::map<std::string, std::map<TuneKey, int>> g_tune;  // per cache file ("" = memory only)

void load_tune_file(const std::string &path, std::map<TuneKey, int> &out) {
  if (path.empty()) return;
  std::ifstream f(path);
  std::string tag;
  int shape, r, cls, m;
  while (f >> tag >> shape >> r >> cls >> m)
    if (tag == "stencil-batched-m") out[TuneKey{shape, r, cls}] = m;
}

void save_tune_file(const std::string &path, const std::map<TuneKey, int> &tab) {
  if (path.empty()) return;
  std::ofstream f(path, std::ios::trunc);
  for (const auto &kv : tab)
    f << "stencil-batched-m " << kv.first.shape << " " << kv.first.r << " " << kv.first.cls
      << " " << kv.second << "\n";
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

// Time m = 1..max_m on a grid of the class's size with the single-grid
// sweep, over enough original steps (a multiple of 8, about 2^27 point-steps)
// that a run lasts far longer than the timer's noise; the fastest of three
// runs per m is compared, and a larger m must win by 3% (ties go to the
// smaller m).
int tune_one(stencil_plan p, int side, int max_m, hipStream_t stream, int *best_m) {
  const size_t bytes = (size_t)side * side * sizeof(float);
  float *a = nullptr, *b = nullptr;
  STENCIL_HIP_TRY(hipMalloc(&a, bytes));
  hipError_t e = hipMalloc(&b, bytes);
  if (e != hipSuccess) {
    (void)hipFree(a);
    return hip_fail(e, "tune alloc");
  }
  (void)hipMemsetAsync(a, 0, bytes, stream);
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  double best = 1e30;
  *best_m = 1;
  int rc = STENCIL_OK;
  for (int m = 1; m <= max_m && rc == STENCIL_OK; ++m) {
    if (m * p->r > kMaxBatchRadius || side < 2 * m * p->r + 1) break;
    stencil_plan_s tmp = *p;  // same weights, own fold depth and device state
    tmp.dev.clear();
    tmp.batch_w32.clear();
    // time what the batch runs: VECTOR kernels, fused passes where the grid
    // allows them (the batched passes fuse as the single-grid sweep does for
    // radius <= 2)
    tmp.mode = STENCIL_MODE_VECTOR;
    tmp.max_fuse = 0;
    rc = stencil_fold_weights(&tmp, m, nullptr, nullptr);
    if (rc) break;
    stencil_grid g{};
    g.data = a;
    g.scratch = b;
    g.dtype = STENCIL_F32;
    g.dim = 2;
    g.shape[0] = g.shape[1] = side;
    g.stream = stream;
    const int64_t pts = (int64_t)side * side;
    const int64_t T = std::min<int64_t>(512, std::max<int64_t>(16, ((1 << 27) / pts + 7) / 8 * 8));
    rc = stencil_run(&tmp, &g, T);  // warm
    float ms = 1e30f;
    for (int rep = 0; rep < 3 && rc == STENCIL_OK; ++rep) {
      (void)hipEventRecord(e0, stream);
      rc = stencil_run(&tmp, &g, T);
      (void)hipEventRecord(e1, stream);
      (void)hipEventSynchronize(e1);
      float t = 0.f;
      (void)hipEventElapsedTime(&t, e0, e1);
      ms = std::min(ms, t);
    }
    free_plan_devices(&tmp);
    if (rc == STENCIL_OK && ms < best * 0.97) {  // 3% margin, ties to smaller m
      best = ms;
      *best_m = m;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(stream);
  (void)hipFree(a);
  (void)hipFree(b);
  return rc;
}

// ---------------------------------------------------------- batch cache

struct BatchEntry {
  std::string key;
  int device = 0;
  Tile *d_tiles_tb = nullptr;  // fused strips (one block each), by group
  int tb_off[kTbGroups + 1] = {0, 0, 0, 0, 0};
  int launches_tb = 0;
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

hipError_t enqueue(const BatchEntry &b, hipStream_t s) {
  for (int k = 0; k < b.launches_tb; ++k) {
    for (int grp = 0; grp < kTbGroups; ++grp) {
      const int n = b.tb_off[grp + 1] - b.tb_off[grp];
      if (n == 0) continue;
      const Tile *t = b.d_tiles_tb + b.tb_off[grp];
      switch (grp) {
        case 0: hipLaunchKernelGGL((k_batched_tb<1, false>), dim3(n), dim3(64), 0, s, t, b.d_grids, b.d_w, k); break;
        case 1: hipLaunchKernelGGL((k_batched_tb<1, true>), dim3(n), dim3(64), 0, s, t, b.d_grids, b.d_w, k); break;
        case 2: hipLaunchKernelGGL((k_batched_tb<2, false>), dim3(n), dim3(64), 0, s, t, b.d_grids, b.d_w, k); break;
        default: hipLaunchKernelGGL((k_batched_tb<2, true>), dim3(n), dim3(64), 0, s, t, b.d_grids, b.d_w, k); break;
      }
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
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

}  // namespace

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

  // --- fold depth per grid: tuned per (shape, r, size class), cached
  std::map<TuneKey, int> &tab = g_tune[cache_path];
  if (tab.empty()) load_tune_file(cache_path, tab);
  std::vector<int> m_of(count, 1);
  bool tuned_any = false;
  for (int i = 0; i < count; ++i) {
    const stencil_plan p = plans[i];
    const int64_t side = std::min(grids[i].shape[0], grids[i].shape[1]);
    const TuneKey key{p->shape, p->r, size_class(side)};
    int m = 1;
    auto it = tab.find(key);
    if (it != tab.end()) {
      m = it->second;
    } else if (autotune) {
      // a representative of the class that runs as the batch will: sides of
      // 256 and more fuse their passes in the batch, so time a vector-aligned
      // side (which the single-grid sweep fuses too)
      int rep_side = (int)std::min<int64_t>(side, 1 << 12);
      if (rep_side >= 256) rep_side = (rep_side + 3) / 4 * 4;
      int rc = tune_one(p, rep_side, max_m, stream, &m);
      if (rc) return rc;
      tab[key] = m;
      tuned_any = true;
    }
    m = std::max(1, std::min(m, max_m));
    while (m > 1 && (m * p->r > kMaxBatchRadius || 2 * m * p->r + 1 > side)) --m;
    m_of[i] = m;
  }
  if (tuned_any) save_tune_file(cache_path, tab);
  if (opts && opts->chosen_m)
    for (int i = 0; i < count; ++i) opts->chosen_m[i] = m_of[i];

  // --- signature of this batch (pointers, sizes, plans, fold depths, T)
  std::ostringstream sig;
  sig << device << ":" << T << ":" << (use_graph ? 1 : 0) << ":" << (uintptr_t)stream;
  for (int i = 0; i < count; ++i)
    sig << "|" << (uintptr_t)plans[i] << "," << (uintptr_t)grids[i].data << ","
        << (uintptr_t)grids[i].scratch << "," << grids[i].shape[0] << "x" << grids[i].shape[1]
        << "," << m_of[i];
  const std::string key = sig.str();
  auto hit = std::find_if(g_cache.begin(), g_cache.end(),
                          [&](const BatchEntry &b) { return b.key == key; });
  if (hit == g_cache.end()) {
    BatchEntry b;
    b.key = key;
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
    std::vector<int> odd;
    int launches = 0, launches_tb = 0;
    for (int i = 0; i < count; ++i) {
      const stencil_plan p = plans[i];
      const stencil_grid &g = grids[i];
      const int m = m_of[i];
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
      // grids of >= 256 vector-aligned columns, up to tb_kmax(R) per pass
      G.fpass = G.nfull = G.tail = 0;
      if (G.nx >= 256 && R <= kMaxBatchRadius && G.ny >= 2 * tb_kmax(R) * R + 1) {
        const int apps = m > 1 ? G.q : G.s;
        const int rest = m > 1 ? G.s : 0;
        const int KM = tb_kmax(R);
        if (apps > 1) {
          // full passes, then the remainder.  An odd launch count is not
          // made even by splitting a pass: a pass costs about the same time
          // whatever its K (it is bound by the strips' memory latency),
          // more than copying the grid back
          G.nfull = apps / KM;
          G.tail = apps % KM;
          G.fpass = G.nfull + (G.tail > 0);
          G.q = 0;
          G.s = rest;
        }
      }
      const int sweeps = G.fpass + (G.fpass ? G.s : G.q + G.s);
      b.passes.push_back(sweeps);
      launches = std::max(launches, G.fpass ? G.s : G.q + G.s);
      launches_tb = std::max(launches_tb, G.fpass);
      if (sweeps % 2) odd.push_back(i);
      if (G.fpass) {
        constexpr int kWout1 = 256 - 2 * tb_border(tb_kmax(1), 1);
        constexpr int kWout2 = 256 - 2 * tb_border(tb_kmax(2), 2);
        const int wout = R == 1 ? kWout1 : kWout2;
        const int kk = G.nfull ? tb_kmax(R) : G.tail;
        const int rows = tb_rows();
        for (int y0 = 0; y0 < G.ny; y0 += rows)
          for (int x0 = 0; x0 < G.nx; x0 += wout) {
            const int y1 = std::min(G.ny, y0 + rows);
            const int64_t cost = (int64_t)(y1 - y0 + 2 * kk * R) * kk * (2 * R + 1);
            tiles_tb[(R - 1) * 2 + (vx4 ? 1 : 0)].push_back({cost, Tile{i, x0, y0, y1}});
          }
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
    b.launches_tb = tltb.empty() ? 0 : launches_tb;
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
