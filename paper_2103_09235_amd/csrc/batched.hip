// Batched sweeps: many independent 2D grids of uneven sizes and mixed
// stencils advanced together.
//
// Small grids waste a GPU when launched one by one (a 64 x 64 grid is 16 KB
// of traffic, far below a launch's fixed cost).  Here every (folded) sweep
// of every grid is one persistent launch: the host cuts all grids into tiles
// (one wavefront streams one tile, as in the single-grid 2D sweep), sorts
// them by decreasing cost, and each workgroup takes tiles round-robin,
// branching per tile (never per lane) to the kernel variant of that grid's
// operator.  The ceil(T/m)-ish launches of the time loop, plus one copy for
// grids whose sweep count is odd, are captured once in a hipGraph and
// replayed.  The fold depth m of each grid is chosen per (stencil, size
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
    if (k >= g.q + g.s) continue;
    const bool folded = k < g.q;
    const int var = folded ? g.var_f : g.var_p;
    const WPtr<float> w{wtab + (folded ? g.w_f : g.w_p)};
    const float *in = (k & 1) ? g.scratch : g.data;
    float *out = (k & 1) ? g.data : g.scratch;
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
// sweep, T = 4 * lcm-free multiple; the fastest per original step wins, ties
// to the smaller m.
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
    // the batched kernel applies the operator once per launch: time that
    tmp.mode = STENCIL_MODE_VECTOR;
    tmp.max_fuse = 1;
    rc = stencil_fold_weights(&tmp, m, nullptr, nullptr);
    if (rc) break;
    stencil_grid g{};
    g.data = a;
    g.scratch = b;
    g.dtype = STENCIL_F32;
    g.dim = 2;
    g.shape[0] = g.shape[1] = side;
    g.stream = stream;
    const int64_t T = 8;
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
    if (rc == STENCIL_OK && ms < best * 0.98) {  // 2% margin, ties to smaller m
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
  Tile *d_tiles = nullptr;
  GridInfo *d_grids = nullptr;
  float *d_w = nullptr;
  int *d_odd = nullptr;
  int ntiles = 0, nodd = 0, launches = 0, nblocks = 0;
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
  if (b.d_grids) (void)hipFree(b.d_grids);
  if (b.d_w) (void)hipFree(b.d_w);
  if (b.d_odd) (void)hipFree(b.d_odd);
  (void)hipSetDevice(cur);
}

hipError_t enqueue(const BatchEntry &b, hipStream_t s) {
  for (int k = 0; k < b.launches; ++k) {
    hipLaunchKernelGGL(k_batched, dim3(b.nblocks), dim3(64), 0, s, b.d_tiles, b.ntiles,
                       b.d_grids, b.d_w, k);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (b.nodd > 0) {
    hipLaunchKernelGGL(k_batched_copyback, dim3(64, std::min(b.nodd, 4096)), dim3(256), 0, s,
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
      const int rep_side = (int)std::min<int64_t>(side, 1 << 12);
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
    std::vector<std::pair<int64_t, Tile>> tiles;
    std::vector<int> odd;
    int launches = 0;
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
      const int sweeps = G.q + G.s;
      launches = std::max(launches, sweeps);
      if (sweeps % 2) odd.push_back(i);
      const int bx = 256;
      const int R = m * p->r;
      for (int y0 = 0; y0 < G.ny; y0 += kTileRows)
        for (int x0 = 0; x0 < G.nx; x0 += bx) {
          const int y1 = std::min(G.ny, y0 + kTileRows);
          const int64_t cost = (int64_t)(y1 - y0 + 2 * R) * (2 * R + 1);
          tiles.push_back({cost, Tile{i, x0, y0, y1}});
        }
    }
    std::stable_sort(tiles.begin(), tiles.end(),
                     [](const auto &a, const auto &b) { return a.first > b.first; });
    std::vector<Tile> tl(tiles.size());
    for (size_t t = 0; t < tiles.size(); ++t) tl[t] = tiles[t].second;
    b.ntiles = (int)tl.size();
    b.nodd = (int)odd.size();
    b.launches = launches;
    hipDeviceProp_t prop;
    STENCIL_HIP_TRY(hipGetDeviceProperties(&prop, device));
    b.nblocks = std::max(1, std::min(b.ntiles, prop.multiProcessorCount * 32));
    hipError_t e = hipMalloc(&b.d_tiles, sizeof(Tile) * tl.size());
    if (e == hipSuccess) e = hipMalloc(&b.d_grids, sizeof(GridInfo) * gi.size());
    if (e == hipSuccess) e = hipMalloc(&b.d_w, sizeof(float) * std::max<size_t>(1, wt.size()));
    if (e == hipSuccess) e = hipMalloc(&b.d_odd, sizeof(int) * std::max<size_t>(1, odd.size()));
    if (e == hipSuccess) e = hipMemcpy(b.d_tiles, tl.data(), sizeof(Tile) * tl.size(), hipMemcpyHostToDevice);
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
  return STENCIL_OK;
}
