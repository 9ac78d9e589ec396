// C ABI of libstencil.so: plan management, validation, the time loop and
// its buffer parity.  Every entry point validates before any device work and
// returns a status; no exception leaves this file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <sstream>
#include <string>

#include "internal.h"

namespace stencil {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

int fail(int code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? STENCIL_E_NOMEM : STENCIL_E_DEVICE;
}

namespace {

constexpr int kMaxFoldedRadius = 64;
constexpr int64_t kMaxWeights = 1 << 20;

size_t esize(int dtype) { return dtype == STENCIL_F64 ? 8 : 4; }

bool on_axes(int64_t idx, int dim, int r) {
  const int s = 2 * r + 1;
  int nonzero = 0;
  for (int a = 0; a < dim; ++a) {
    if ((int)(idx % s) != r) ++nonzero;
    idx /= s;
  }
  return nonzero <= 1;
}

void free_operator(OperatorDev &op) {
  if (op.w_dev) (void)hipFree(op.w_dev);
  if (op.taps_dev) (void)hipFree(op.taps_dev);
  if (op.mfma_b) (void)hipFree(op.mfma_b);
  op = OperatorDev();
}

// The plan's run graphs on the current device.  A run using one must not be
// in flight (plans are not mutated while their work is in flight).
void drop_graphs(DeviceState &d) {
  for (auto &kv : d.graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto &kv : d.graph_src) (void)hipGraphDestroy(kv.second);
  d.graphs.clear();
  d.graph_src.clear();
}

void free_device_state(DeviceState &d) {
  free_operator(d.plain32);
  free_operator(d.plain64);
  free_operator(d.fold32);
  free_operator(d.fold64);
  drop_graphs(d);
  if (d.scratch) (void)hipFree(d.scratch);
  d.scratch = nullptr;
  d.scratch_bytes = 0;
  for (void *&b : d.dir_buf) {
    if (b) (void)hipFree(b);
    b = nullptr;
  }
  d.dir_bytes = 0;
  d.ready32 = d.ready64 = false;
  d.ready_m = 0;
}

// Build one operator on the current device from dense host weights.
template <typename T>
int build_operator(const std::vector<T> &w, int dim, int R, int mask,
                   OperatorDev &op) {
  free_operator(op);
  op.R = R;
  op.mask = mask;
  const int s = 2 * R + 1;
  std::vector<int4> taps;
  for (int64_t i = 0; i < (int64_t)w.size(); ++i) {
    if (w[i] == T(0)) continue;
    int o[3] = {0, 0, 0};
    int64_t t = i;
    for (int a = dim - 1; a >= 0; --a) {
      o[3 - dim + a] = (int)(t % s) - R;
      t /= s;
    }
    taps.push_back(int4{o[0], o[1], o[2], (int)i});
  }
  op.ntaps = (int)taps.size();
  STENCIL_HIP_TRY(hipMalloc(&op.w_dev, sizeof(T) * w.size()));
  STENCIL_HIP_TRY(hipMemcpy(op.w_dev, w.data(), sizeof(T) * w.size(),
                            hipMemcpyHostToDevice));
  STENCIL_HIP_TRY(hipMalloc(&op.taps_dev, sizeof(int4) * std::max<size_t>(1, taps.size())));
  if (!taps.empty())
    STENCIL_HIP_TRY(hipMemcpy(op.taps_dev, taps.data(), sizeof(int4) * taps.size(),
                              hipMemcpyHostToDevice));
  if (dim == 2) {
    op.symmetric = true;
    for (int a = 0; a < s && op.symmetric; ++a)
      for (int b = 0; b < s; ++b) {
        const T v = w[(size_t)a * s + b];
        if (v != w[(size_t)a * s + (s - 1 - b)] || v != w[(size_t)(s - 1 - a) * s + b]) {
          op.symmetric = false;
          break;
        }
      }
  }
  if constexpr (sizeof(T) == 4) {
    op.w32.assign(w.begin(), w.end());
    if (dim == 2 && R <= 8) {
      const std::vector<uint16_t> t = mfma_b_table(op.w32, R);
      STENCIL_HIP_TRY(hipMalloc(&op.mfma_b, t.size() * sizeof(uint16_t)));
      STENCIL_HIP_TRY(hipMemcpy(op.mfma_b, t.data(), t.size() * sizeof(uint16_t),
                                hipMemcpyHostToDevice));
    }
  } else {
    op.w64.assign(w.begin(), w.end());
  }
  return STENCIL_OK;
}

// Operators for the current fold depth and dtype on the current device.
// The separable form of a 2D operator W (FP64, side S): its rank (up to S)
// and whether mode SEPARABLE applies it: rank 1 or 2 and 2 * rank * S FMAs
// per point fewer than W's nonzero taps.
bool separable_form(const std::vector<double> &W, int S, int *rank_out,
                    std::vector<double> *a, std::vector<double> *b) {
  std::vector<double> fa, fb;
  const int rank = low_rank_2d(W, S, S, fa, fb);
  int taps = 0;
  for (double v : W) taps += v != 0.0;
  if (rank_out) *rank_out = rank;
  if (a) *a = fa;
  if (b) *b = fb;
  return rank >= 1 && rank <= 2 && 2 * rank * S < taps;
}

// A 3D operator of tensor rank one, a (x) b (x) c, cheaper as three 1D passes
// (3(2R+1) FMAs) than as its nonzero taps.
bool separable_form_3d(const std::vector<double> &W, int S, std::vector<double> *f) {
  std::vector<double> a, b, c;
  if (!product_3d(W, S, a, b, c)) return false;
  int taps = 0;
  for (double v : W) taps += v != 0.0;
  if (3 * S >= taps) return false;
  if (f) {
    *f = a;
    f->insert(f->end(), b.begin(), b.end());
    f->insert(f->end(), c.begin(), c.end());
  }
  return true;
}

void attach_separable_3d(const std::vector<double> &W, int R, OperatorDev &op) {
  const int S = 2 * R + 1;
  std::vector<double> f;
  op.sep_rank = 0;
  op.sep32.clear();
  if (!separable_form_3d(W, S, &f)) return;
  round_factors_f32(f, S, op.sep32);
  op.sep_rank = 1;
}

void attach_separable(const std::vector<double> &W, int R, OperatorDev &op) {
  const int S = 2 * R + 1;
  std::vector<double> a, b;
  int rank = 0;
  op.sep_rank = 0;
  op.sep32.clear();
  if (!separable_form(W, S, &rank, &a, &b)) return;
  std::vector<double> f = a;
  f.insert(f.end(), b.begin(), b.end());
  round_factors_f32(f, S, op.sep32);
  op.sep_rank = rank;
}

int ensure_operators(stencil_plan p, int device, int dtype) {
  DeviceState &d = p->dev[device];
  if (d.ready_m != p->m) {
    d.ready32 = d.ready64 = false;
    d.ready_m = p->m;
  }
  // graphs hold the operators' device pointers and weights
  if ((dtype == STENCIL_F32 && !d.ready32) || (dtype == STENCIL_F64 && !d.ready64)) drop_graphs(d);
  const int R = p->m * p->r;
  if (dtype == STENCIL_F32 && !d.ready32) {
    std::vector<float> w32(p->w.size());
    for (size_t i = 0; i < w32.size(); ++i) w32[i] = (float)p->w[i];
    int rc = build_operator(w32, p->dim, p->r, mask_for(p->shape, 1), d.plain32);
    if (rc) return rc;
    rc = build_operator(p->Wm32, p->dim, R, mask_for(p->shape, p->m), d.fold32);
    if (rc) return rc;
    if (p->dim == 2) {
      attach_separable(p->w, p->r, d.plain32);
      attach_separable(p->Wm, R, d.fold32);
    } else if (p->dim == 3) {
      attach_separable_3d(p->w, p->r, d.plain32);
      attach_separable_3d(p->Wm, R, d.fold32);
    }
    d.ready32 = true;
  }
  if (dtype == STENCIL_F64 && !d.ready64) {
    int rc = build_operator(p->w, p->dim, p->r, mask_for(p->shape, 1), d.plain64);
    if (rc) return rc;
    rc = build_operator(p->Wm, p->dim, R, mask_for(p->shape, p->m), d.fold64);
    if (rc) return rc;
    d.ready64 = true;
  }
  return STENCIL_OK;
}

hipError_t dispatch(stencil_plan p, const SweepLaunch &L) {
  if (p->mode == STENCIL_MODE_EXACT_ORDER) return launch_naive(L);
  if (p->mode == STENCIL_MODE_MFMA_BF16X3) return launch_mfma2d(L);
  hipError_t e = hipErrorNotSupported;
  if (L.g.dim == 1) e = launch_sweep1d(L);
  else if (L.g.dim == 2) {
    SweepLaunch Ls = L;
    Ls.sym = p->mode == STENCIL_MODE_SYMMETRIC;
    Ls.sep = p->mode == STENCIL_MODE_SEPARABLE;
    e = L.steps > 1 ? launch_sweep2d_tb(Ls) : launch_sweep2d(Ls);
  }
  else if (p->mode == STENCIL_MODE_SEPARABLE && L.steps == 1 && L.op->sep_rank == 1)
    e = launch_sweep3d_sep(L);
  else e = L.steps > 1 ? launch_sweep3d_tb(L) : launch_sweep3d(L);
  if (e == hipErrorNotSupported) {
    // the generic kernel neither fuses steps nor applies a floor
    if (L.steps != 1 || L.floor) return hipErrorNotSupported;
    (void)hipGetLastError();
    e = launch_naive(L);
  }
  return e;
}

int check_plan(stencil_plan p) {
  if (!p) return fail(STENCIL_E_ARG, "plan is NULL");
  return STENCIL_OK;
}

}  // namespace

void free_plan_devices(stencil_plan_s *p) {
  int cur = 0;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  for (auto &kv : p->dev)
    if (hipSetDevice(kv.first) == hipSuccess) free_device_state(kv.second);
  p->dev.clear();
  if (have) (void)hipSetDevice(cur);
}

void drop_plan_graphs(stencil_plan_s *p) {
  int cur = 0;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  for (auto &kv : p->dev)
    if (!kv.second.graphs.empty() && hipSetDevice(kv.first) == hipSuccess) drop_graphs(kv.second);
  if (have) (void)hipSetDevice(cur);
}

}  // namespace stencil

using namespace stencil;

extern "C" {

const char *stencil_last_error(void) { return g_last_error.c_str(); }

const char *stencil_version(void) { return "stencilfold 0.1.0 (gfx950)"; }

int stencil_plan_create(int dim, int radius, int shape, const double *weights,
                        int boundary, stencil_plan *out) {
  set_error("");
  if (!out) return fail(STENCIL_E_ARG, "out is NULL");
  *out = nullptr;
  if (dim < 1 || dim > 3) return fail(STENCIL_E_ARG, "dim must be 1, 2 or 3");
  if (radius < 1) return fail(STENCIL_E_ARG, "radius must be >= 1");
  if (radius > kMaxFoldedRadius)
    return fail(STENCIL_E_UNSUPPORTED, "radius too large");
  if (shape != STENCIL_STAR && shape != STENCIL_BOX)
    return fail(STENCIL_E_ARG, "shape must be STENCIL_STAR or STENCIL_BOX");
  if (boundary != STENCIL_PERIODIC && boundary != STENCIL_DIRICHLET)
    return fail(STENCIL_E_ARG, "boundary must be PERIODIC or DIRICHLET");
  if (!weights) return fail(STENCIL_E_ARG, "weights is NULL");
  const int64_t n = count_of(dim, radius);
  if (n > kMaxWeights) return fail(STENCIL_E_UNSUPPORTED, "stencil too large");
  for (int64_t i = 0; i < n; ++i) {
    if (!std::isfinite(weights[i])) return fail(STENCIL_E_ARG, "weights must be finite");
    if (shape == STENCIL_STAR && weights[i] != 0.0 && !on_axes(i, dim, radius))
      return fail(STENCIL_E_ARG, "STAR stencil has a nonzero weight off the axes");
  }
  stencil_plan p = new (std::nothrow) stencil_plan_s();
  if (!p) return fail(STENCIL_E_NOMEM, "plan allocation failed");
  static std::atomic<uint64_t> next_id{1};
  p->id = next_id.fetch_add(1);
  try {
    p->dim = dim;
    p->r = radius;
    p->shape = shape;
    p->boundary = boundary;
    p->w.assign(weights, weights + n);
    p->m = 1;
    p->Wm = p->w;
    round_fold_f32(p->w, p->Wm, dim, radius, 1, p->Wm32);
    p->Wm_hi.resize(n);
    p->Wm_lo.resize(n);
    for (int64_t i = 0; i < n; ++i) {
      p->Wm_hi[i] = bf16_rne(p->Wm32[i]);
      float hi;
      uint32_t b = (uint32_t)p->Wm_hi[i] << 16;
      std::memcpy(&hi, &b, 4);
      p->Wm_lo[i] = bf16_rne(p->Wm32[i] - hi);
    }
  } catch (...) {
    delete p;
    return fail(STENCIL_E_NOMEM, "plan allocation failed");
  }
  *out = p;
  return STENCIL_OK;
}

int stencil_fold_weights(stencil_plan p, int m, double *out_or_null,
                         int64_t *out_len) {
  set_error("");
  if (int rc = check_plan(p)) return rc;
  if (m < 1) return fail(STENCIL_E_ARG, "m must be >= 1");
  if ((int64_t)m * p->r > kMaxFoldedRadius)
    return fail(STENCIL_E_UNSUPPORTED, "folded radius m*r too large");
  const int R = m * p->r;
  const int64_t n = count_of(p->dim, R);
  if (n > kMaxWeights) return fail(STENCIL_E_UNSUPPORTED, "folded stencil too large");
  std::vector<double> Wm;
  std::vector<float> W32;
  std::vector<uint16_t> hi(n), lo(n);
  try {
    int rc = fold_on_device(p->w, p->dim, p->r, m, Wm);
    if (rc) return rc;
    round_fold_f32(p->w, Wm, p->dim, R, m, W32);
    for (int64_t i = 0; i < n; ++i) {
      hi[i] = bf16_rne(W32[i]);
      float h;
      uint32_t b = (uint32_t)hi[i] << 16;
      std::memcpy(&h, &b, 4);
      lo[i] = bf16_rne(W32[i] - h);
    }
  } catch (...) {
    return fail(STENCIL_E_NOMEM, "host allocation failed");
  }
  drop_plan_graphs(p);
  p->m = m;
  p->Wm.swap(Wm);
  p->Wm32.swap(W32);
  p->Wm_hi.swap(hi);
  p->Wm_lo.swap(lo);
  if (out_or_null) std::memcpy(out_or_null, p->Wm.data(), sizeof(double) * n);
  if (out_len) *out_len = n;
  return STENCIL_OK;
}

int stencil_fold_weights_f32(stencil_plan p, float *out, int64_t *out_len) {
  set_error("");
  if (int rc = check_plan(p)) return rc;
  if (out) std::memcpy(out, p->Wm32.data(), sizeof(float) * p->Wm32.size());
  if (out_len) *out_len = (int64_t)p->Wm32.size();
  return STENCIL_OK;
}

int stencil_plan_set_mode(stencil_plan p, int mode) {
  set_error("");
  if (int rc = check_plan(p)) return rc;
  if (mode != STENCIL_MODE_VECTOR && mode != STENCIL_MODE_EXACT_ORDER &&
      mode != STENCIL_MODE_MFMA_BF16X3 && mode != STENCIL_MODE_SYMMETRIC &&
      mode != STENCIL_MODE_SEPARABLE)
    return fail(STENCIL_E_ARG, "unknown mode");
  if (mode == STENCIL_MODE_SYMMETRIC && p->dim != 2)
    return fail(STENCIL_E_UNSUPPORTED, "SYMMETRIC mode needs a 2D plan");
  if (mode == STENCIL_MODE_SEPARABLE && p->dim == 1)
    return fail(STENCIL_E_UNSUPPORTED, "SEPARABLE mode needs a 2D or 3D plan");
  if (mode == STENCIL_MODE_MFMA_BF16X3 && p->dim != 2)
    return fail(STENCIL_E_UNSUPPORTED, "MFMA mode needs a 2D plan");
  drop_plan_graphs(p);
  p->mode = mode;
  return STENCIL_OK;
}

int stencil_plan_separable(stencil_plan p, int *rank, int *applies) {
  set_error("");
  if (int rc = check_plan(p)) return rc;
  const int R = p->m * p->r;
  if (p->dim == 3) {
    const bool ok = separable_form_3d(p->m > 1 ? p->Wm : p->w, 2 * R + 1, nullptr);
    std::vector<double> a, b, c;
    if (rank) *rank = product_3d(p->m > 1 ? p->Wm : p->w, 2 * R + 1, a, b, c) ? 1 : 0;
    if (applies) *applies = ok ? 1 : 0;
    return STENCIL_OK;
  }
  if (p->dim != 2) {
    if (rank) *rank = 0;
    if (applies) *applies = 0;
    return STENCIL_OK;
  }
  const bool ok = separable_form(p->m > 1 ? p->Wm : p->w, 2 * R + 1, rank, nullptr, nullptr);
  if (applies) *applies = ok ? 1 : 0;
  return STENCIL_OK;
}

int stencil_plan_set_floor(stencil_plan p, const void *floor, int dtype, int64_t count) {
  set_error("");
  if (int rc = check_plan(p)) return rc;
  if (!floor) {
    drop_plan_graphs(p);
    p->floor = nullptr;
    p->floor_count = 0;
    return STENCIL_OK;
  }
  if (dtype != STENCIL_F32 && dtype != STENCIL_F64)
    return fail(STENCIL_E_ARG, "dtype must be STENCIL_F32 or STENCIL_F64");
  if (count < 1) return fail(STENCIL_E_ARG, "count must be >= 1");
  if (p->dim != 1 || p->r > 8)
    return fail(STENCIL_E_UNSUPPORTED, "a floor needs a 1D plan of radius <= 8");
  if (p->boundary != STENCIL_PERIODIC)
    return fail(STENCIL_E_UNSUPPORTED, "a floor needs periodic boundaries");
  drop_plan_graphs(p);
  p->floor = floor;
  p->floor_dtype = dtype;
  p->floor_count = count;
  return STENCIL_OK;
}

namespace stencil {
namespace {
// The generations of each launch of a Game of Life run: the largest of 16,
// 8, 4, 2 allowed, else 1.
std::vector<int> life_schedule(int64_t ny, int64_t nx, const void *a, const void *b, int64_t T) {
  std::vector<int> ks;
  const int kmax = life_max_steps(ny, nx, a, b);
  for (int64_t left = T; left > 0;) {
    int k = 1;
    for (int c = 16; c >= 2; c /= 2)
      if (c <= kmax && c <= left && 2 * c + 1 <= ny) {
        k = c;
        break;
      }
    ks.push_back(k);
    left -= k;
  }
  return ks;
}
}  // namespace
}  // namespace stencil

int stencil_life_launches(int64_t ny, int64_t nx, int64_t T, int64_t *launches) {
  set_error("");
  if (ny < 1 || nx < 1 || T < 0 || !launches) return fail(STENCIL_E_ARG, "bad arguments");
  // caller buffers from hipMalloc are 4-byte aligned
  *launches = (int64_t)life_schedule(ny, nx, (void *)16, (void *)32, T).size();
  return STENCIL_OK;
}

int stencil_life(void *cells, void *scratch, int64_t ny, int64_t nx, int64_t T, void *stream) {
  set_error("");
  if (!cells || !scratch) return fail(STENCIL_E_ARG, "cells and scratch must be non-NULL");
  if (ny < 1 || nx < 1) return fail(STENCIL_E_ARG, "ny and nx must be >= 1");
  if (T < 0) return fail(STENCIL_E_ARG, "T must be >= 0");
  if (ny > ((int64_t)1 << 30) || nx > ((int64_t)1 << 30) || ny * nx > ((int64_t)1 << 40))
    return fail(STENCIL_E_UNSUPPORTED, "grid too large");
  const int64_t bytes = ny * nx;
  const char *a = (const char *)cells, *b = (const char *)scratch;
  if (a < b + bytes && b < a + bytes) return fail(STENCIL_E_ARG, "cells and scratch overlap");
  if (T == 0) return STENCIL_OK;
  hipStream_t s = (hipStream_t)stream;
  const uint8_t *src = (const uint8_t *)cells;
  uint8_t *dst = (uint8_t *)scratch;
  // generations in fused launches of 16, 8, 4 or 2 where the grid allows,
  // the rest one per launch
  for (int k : life_schedule(ny, nx, cells, scratch, T)) {
    hipError_t e = k > 1 ? launch_life_fused(src, dst, ny, nx, k, s)
                         : launch_life(src, dst, ny, nx, s);
    if (e != hipSuccess) return hip_fail(e, "life generation");
    const uint8_t *o = src;
    src = dst;
    dst = const_cast<uint8_t *>(o);
  }
  if (src != cells) {
    hipError_t e = launch_copy(src, cells, bytes, s);
    if (e != hipSuccess) return hip_fail(e, "final copy");
  }
  return STENCIL_OK;
}

int stencil_plan_set_fusion(stencil_plan p, int max_steps) {
  set_error("");
  if (int rc = check_plan(p)) return rc;
  if (max_steps < 0) return fail(STENCIL_E_ARG, "max_steps must be >= 0");
  drop_plan_graphs(p);
  p->max_fuse = max_steps;
  return STENCIL_OK;
}

int stencil_plan_set_boundary_value(stencil_plan p, double value) {
  set_error("");
  if (int rc = check_plan(p)) return rc;
  if (!std::isfinite(value)) return fail(STENCIL_E_ARG, "the boundary value must be finite");
  if (p->boundary != STENCIL_DIRICHLET && value != 0.0)
    return fail(STENCIL_E_UNSUPPORTED, "a boundary value needs a STENCIL_DIRICHLET plan");
  p->bvalue = value;
  return STENCIL_OK;
}

int stencil_plan_set_graph(stencil_plan p, int on) {
  set_error("");
  if (int rc = check_plan(p)) return rc;
  if (on != 0 && on != 1) return fail(STENCIL_E_ARG, "on must be 0 or 1");
  if (!on) drop_plan_graphs(p);
  p->use_graph = on;
  return STENCIL_OK;
}

int stencil_plan_info(stencil_plan p, int *dim, int *radius, int *m,
                      int *folded_radius, int *mode) {
  set_error("");
  if (int rc = check_plan(p)) return rc;
  if (dim) *dim = p->dim;
  if (radius) *radius = p->r;
  if (m) *m = p->m;
  if (folded_radius) *folded_radius = p->m * p->r;
  if (mode) *mode = p->mode;
  return STENCIL_OK;
}

int stencil_profitability(stencil_plan p, int m, int64_t *naive, int64_t *folded) {
  set_error("");
  if (int rc = check_plan(p)) return rc;
  if (m < 1) return fail(STENCIL_E_ARG, "m must be >= 1");
  if ((int64_t)m * p->r > kMaxFoldedRadius)
    return fail(STENCIL_E_UNSUPPORTED, "m*r too large");
  try {
    profitability(p->w, p->dim, p->r, m, naive, folded);
  } catch (...) {
    return fail(STENCIL_E_NOMEM, "host allocation failed");
  }
  return STENCIL_OK;
}

namespace stencil {
namespace {

// Checks a run's arguments (no device work) and fills its geometry.
int check_run(stencil_plan p, const stencil_grid *g, int64_t T, Geom &geo) {
  if (int rc = check_plan(p)) return rc;
  if (!g) return fail(STENCIL_E_ARG, "grid is NULL");
  if (T < 0) return fail(STENCIL_E_ARG, "T must be >= 0");
  if (g->dim != p->dim) return fail(STENCIL_E_ARG, "grid dim differs from plan dim");
  if (g->dtype != STENCIL_F32 && g->dtype != STENCIL_F64)
    return fail(STENCIL_E_ARG, "dtype must be STENCIL_F32 or STENCIL_F64");
  if (!g->data) return fail(STENCIL_E_ARG, "data is NULL");
  if (p->mode == STENCIL_MODE_MFMA_BF16X3 && g->dtype != STENCIL_F32)
    return fail(STENCIL_E_UNSUPPORTED, "MFMA mode takes FP32 grids only");
  if (p->mode == STENCIL_MODE_MFMA_BF16X3 && p->m * p->r > 8)
    return fail(STENCIL_E_UNSUPPORTED, "MFMA mode needs a folded radius m*r <= 8");
  geo = Geom();
  geo.dim = p->dim;
  int64_t n[3] = {1, 1, 1};
  for (int a = 0; a < p->dim; ++a) {
    if (g->shape[a] < 1) return fail(STENCIL_E_ARG, "grid axes must be >= 1");
    n[3 - p->dim + a] = g->shape[a];
  }
  geo.nz = n[0];
  geo.ny = n[1];
  geo.nx = n[2];
  // periodic runs wrap once at most; zero-boundary runs pad the grid
  const int64_t need = p->boundary == STENCIL_PERIODIC ? 2 * (int64_t)p->m * p->r + 1 : 1;
  for (int a = 0; a < p->dim; ++a)
    if (g->shape[a] < need)
      return fail(STENCIL_E_UNSUPPORTED,
                  "every grid axis must be >= 2*m*r+1 for this plan");
  if (geo.count() > ((int64_t)1 << 40)) return fail(STENCIL_E_UNSUPPORTED, "grid too large");
  if (p->boundary == STENCIL_DIRICHLET) {
    // the fused kernels take the padded grid's interior box (each axis
    // padded by m*r on both sides, rows rounded up to 256 bytes) as int
    const int64_t lim = (int64_t)INT_MAX - 2 * (int64_t)p->m * p->r - 64;
    for (int a = 0; a < p->dim; ++a)
      if (g->shape[a] > lim)
        return fail(STENCIL_E_UNSUPPORTED,
                    "zero-boundary grid axes must be below 2^31 - 2*m*r - 64 points");
  }
  if (p->floor) {
    if (p->m != 1)
      return fail(STENCIL_E_UNSUPPORTED, "a floor makes the update nonlinear: fold depth must be 1");
    if (p->mode != STENCIL_MODE_VECTOR)
      return fail(STENCIL_E_UNSUPPORTED, "a floor runs in VECTOR mode only");
    if (g->dtype != p->floor_dtype || geo.count() != p->floor_count)
      return fail(STENCIL_E_ARG, "the floor must have the grid's dtype and point count");
  }
  const size_t bytes = (size_t)geo.count() * esize(g->dtype);
  if (g->scratch) {
    const char *a = (const char *)g->data, *b = (const char *)g->scratch;
    if (a < b + bytes && b < a + bytes)
      return fail(STENCIL_E_ARG, "data and scratch overlap");
  }
  return STENCIL_OK;
}

// The launches of a run: floor(T/m) applications of the folded operator,
// then T mod m of the plain one.  Tiled kernels may fuse several
// applications of one operator per launch (1D, 2D and 3D temporal blocking);
// the 2D fused kernel needs 16-byte aligned buffers (a plan-owned scratch
// buffer always is).  An odd launch total leaves the result in scratch and
// costs a final copy, unless a fusing pass can split once more.
struct Schedule {
  int64_t apps[2] = {0, 0};      // folded, plain
  int64_t launches[2] = {0, 0};
  bool final_copy = false;
};

// The zero-padded copy a zero-boundary run works on: pad P = m*r on the
// grid's axes, rows rounded up to whole 256-byte lines; np = extents, off =
// the interior's first index per axis (z, y, x).
Geom padded_geom(stencil_plan p, const Geom &geo, int dtype, int64_t np[3], int64_t off[3]) {
  const int64_t P = (int64_t)p->m * p->r;
  const int64_t n[3] = {geo.nz, geo.ny, geo.nx};
  for (int a = 0; a < 3; ++a) {
    const bool axis = a >= 3 - p->dim;
    off[a] = axis ? P : 0;
    np[a] = axis ? n[a] + 2 * P : 1;
  }
  const int64_t line = 256 / (int64_t)esize(dtype);
  np[2] = (np[2] + line - 1) / line * line;
  Geom pg;
  pg.dim = p->dim;
  pg.nz = np[0];
  pg.ny = np[1];
  pg.nx = np[2];
  return pg;
}

Schedule make_schedule(stencil_plan p, const Geom &geo, int dtype, const void *data,
                       const void *scratch, int64_t T) {
  Schedule sc;
  sc.apps[0] = p->m > 1 ? T / p->m : 0;
  sc.apps[1] = p->m > 1 ? T % p->m : T;
  const bool aligned = (uintptr_t)data % 16 == 0 && (uintptr_t)scratch % 16 == 0 &&
                       p->boundary == STENCIL_PERIODIC;
  int64_t kmax[2] = {1, 1};
  for (int i = 0; i < 2; ++i) {
    if (sc.apps[i] == 0) continue;
    OperatorDev op;
    op.R = i == 0 ? p->m * p->r : p->r;
    op.mask = mask_for(p->shape, i == 0 ? p->m : 1);
    SweepLaunch L;
    L.g = geo;
    L.dtype = dtype;
    L.op = &op;
    if (p->boundary != STENCIL_PERIODIC) {
      // plain applications of 2D VECTOR plans and of 1D plans (not
      // EXACT_ORDER) fuse on the padded grid, each step writing the ghost
      // value outside the interior; folded ones restore the pad one by one
      kmax[i] = 1;
      if (i == 1 && p->dim == 2 && p->mode == STENCIL_MODE_VECTOR) {
        int64_t np[3], off[3];
        L.g = padded_geom(p, geo, dtype, np, off);
        kmax[i] = std::max(1, sweep2d_max_steps(L));
      } else if (i == 1 && p->dim == 1 && p->mode != STENCIL_MODE_EXACT_ORDER) {
        int64_t np[3], off[3];
        L.g = padded_geom(p, geo, dtype, np, off);
        kmax[i] = std::max(1, sweep1d_max_steps(L));
      }
    } else if (p->dim == 1 && p->mode != STENCIL_MODE_EXACT_ORDER)
      kmax[i] = std::max(1, sweep1d_max_steps(L));
    else if (p->dim == 2 && p->mode == STENCIL_MODE_VECTOR && aligned)
      kmax[i] = std::max(1, sweep2d_max_steps(L));
    else if (p->dim == 3 && p->mode == STENCIL_MODE_VECTOR)
      kmax[i] = std::max(1, sweep3d_max_steps(L));
    if (p->max_fuse > 0) kmax[i] = std::min<int64_t>(kmax[i], p->max_fuse);
    sc.launches[i] = (sc.apps[i] + kmax[i] - 1) / kmax[i];
  }
  // an even launch count saves the final copy (zero-boundary runs always
  // copy the padded result back)
  for (int i = 0; i < 2 && p->boundary == STENCIL_PERIODIC; ++i) {
    if ((sc.launches[0] + sc.launches[1]) % 2 == 0) break;
    if (kmax[i] > 1 && sc.launches[i] < sc.apps[i]) sc.launches[i] += 1;
  }
  sc.final_copy = (sc.launches[0] + sc.launches[1]) % 2 == 1 ||
                  (p->boundary != STENCIL_PERIODIC && T > 0);
  return sc;
}

// A Dirichlet run (reading in dirichlet.hip): the grid is copied into a
// padded buffer whose pad holds the ghost value (pad P = m*r on the grid's
// axes, rows rounded up to whole 256-byte lines), each application runs the
// periodic kernels on the padded grid, then restores the pad; a folded
// application also recomputes the band closer than (m-1)r to a face from m
// plain steps on a frame of width 2(m-1)r.  Plain applications of 2D FP32
// VECTOR plans and of 1D plans fuse several per launch, the fused kernels
// writing the ghost value outside the interior at every stage.  The
// result is copied back into g->data; g->scratch is not used.
int run_dirichlet(stencil_plan p, stencil_grid *g, int64_t T, const Geom &geo, DeviceState &d) {
  const int m = p->m, r = p->r;
  const int dtype = g->dtype;
  const size_t es = esize(dtype);
  const int64_t n[3] = {geo.nz, geo.ny, geo.nx};
  int64_t np[3], off[3];
  // padded rows in whole 256-byte lines (aligned row segments for the tiles)
  const Geom pg = padded_geom(p, geo, dtype, np, off);
  const size_t bytes = (size_t)(np[0] * np[1] * np[2]) * es;
  if (d.dir_bytes < bytes) {
    if (d.dir_bytes) STENCIL_HIP_TRY(hipDeviceSynchronize());
    for (void *&b : d.dir_buf) {
      if (b) (void)hipFree(b);
      b = nullptr;
    }
    d.dir_bytes = 0;
    for (void *&b : d.dir_buf) STENCIL_HIP_TRY(hipMalloc(&b, bytes));
    d.dir_bytes = bytes;
  }
  hipStream_t s = (hipStream_t)g->stream;
  const OperatorDev &plain = dtype == STENCIL_F32 ? d.plain32 : d.plain64;
  const OperatorDev &folded = dtype == STENCIL_F32 ? d.fold32 : d.fold64;
  void *A = d.dir_buf[0], *B = d.dir_buf[1];
  void *F[2] = {d.dir_buf[2], d.dir_buf[3]};
  const int64_t ibase = (off[0] * np[1] + off[1]) * np[2] + off[2];
  hipError_t e = dirichlet_box_copy(g->data, 0, n[1] * n[2], n[2], A, ibase, np[1] * np[2],
                                    np[2], n, dtype, s);
  // pads cleared on every run: the buffers may hold another geometry's data
  for (void *b : {A, F[0], F[1]})
    if (e == hipSuccess) e = dirichlet_clear_pad(b, np, off, n, dtype, p->bvalue, s);
  if (e != hipSuccess) return hip_fail(e, "zero-boundary set-up");
  SweepLaunch L;
  L.g = pg;
  L.dtype = dtype;
  L.stream = s;
  L.steps = 1;
  const Schedule sc = make_schedule(p, geo, dtype, g->data, g->data, T);
  const int64_t q = sc.apps[0];
  const int64_t Wb = (int64_t)(m - 1) * r, Wf = 2 * Wb;
  int64_t left = sc.apps[1];  // plain applications still to launch
  const int64_t nl = q + sc.launches[1];
  for (int64_t k = 0; k < nl; ++k) {
    const bool fold = k < q;
    L.op = fold ? &folded : &plain;
    L.in = A;
    L.out = B;
    L.steps = 1;
    L.zb = false;
    if (!fold) {
      // plain applications spread evenly over the remaining launches
      L.steps = (int)((left + (nl - k) - 1) / (nl - k));
      left -= L.steps;
      if (L.steps > 1) {
        L.zb = true;
        L.zval = p->bvalue;
        L.zbox[0] = (int)off[1];
        L.zbox[1] = (int)(off[1] + n[1]);
        L.zbox[2] = (int)off[2];
        L.zbox[3] = (int)(off[2] + n[2]);
      }
    }
    e = dispatch(p, L);
    if (e == hipSuccess && fold && m > 1) {
      // levels 1 .. m-1 on the frame, level m into the band of B
      const void *src = A;
      for (int j = 1; j < m && e == hipSuccess; ++j) {
        e = dirichlet_frame_step(src, F[(j - 1) & 1], np, off, n, Wf, plain, dtype, s);
        src = F[(j - 1) & 1];
      }
      if (e == hipSuccess) e = dirichlet_frame_step(src, B, np, off, n, Wb, plain, dtype, s);
    }
    // a fused launch leaves the pad zero; the others restore it
    if (e == hipSuccess && !L.zb) e = dirichlet_clear_pad(B, np, off, n, dtype, p->bvalue, s);
    if (e != hipSuccess) return hip_fail(e, "zero-boundary sweep");
    std::swap(A, B);
  }
  e = dirichlet_box_copy(A, ibase, np[1] * np[2], np[2], g->data, 0, n[1] * n[2], n[2], n, dtype,
                         s);
  if (e != hipSuccess) return hip_fail(e, "zero-boundary copy-back");
  return STENCIL_OK;
}

// The launches of a periodic run on stream s: the schedule's applications,
// the two buffers alternating, and the final copy of an odd launch count.
int enqueue_run(stencil_plan p, const Geom &geo, int dtype, const void *data, void *scratch,
                int64_t T, DeviceState &d, hipStream_t s) {
  const size_t bytes = (size_t)geo.count() * esize(dtype);
  const OperatorDev *ops[2] = {dtype == STENCIL_F32 ? &d.fold32 : &d.fold64,
                               dtype == STENCIL_F32 ? &d.plain32 : &d.plain64};
  const Schedule sc = make_schedule(p, geo, dtype, data, scratch, T);
  SweepLaunch L;
  L.g = geo;
  L.dtype = dtype;
  L.stream = s;
  L.floor = p->floor;
  const void *src = data;
  void *dst = scratch;
  for (int i = 0; i < 2; ++i) {
    if (sc.apps[i] == 0) continue;
    L.op = ops[i];
    int64_t left = sc.apps[i];
    const int64_t nl = sc.launches[i];
    for (int64_t k = 0; k < nl; ++k) {
      const int64_t take = (left + (nl - k) - 1) / (nl - k);
      L.in = src;
      L.out = dst;
      L.steps = (int)take;
      hipError_t e = dispatch(p, L);
      if (e != hipSuccess) return hip_fail(e, "sweep launch");
      left -= take;
      const void *t = src;
      src = dst;
      dst = const_cast<void *>(t);
    }
  }
  if (src != data) {
    hipError_t e = launch_copy(src, const_cast<void *>(data), (int64_t)bytes, s);
    if (e != hipSuccess) return hip_fail(e, "final copy");
  }
  return STENCIL_OK;
}

constexpr size_t kMaxRunGraphs = 16;  // per plan and device
constexpr int64_t kGraphMinLaunches = 4;  // shorter runs are launched directly

}  // namespace
}  // namespace stencil

int stencil_run_schedule(stencil_plan p, const stencil_grid *g, int64_t T, int64_t *out,
                         int *final_copy) {
  set_error("");
  Geom geo;
  if (int rc = check_run(p, g, T, geo)) return rc;
  if (!out) return fail(STENCIL_E_ARG, "out is NULL");
  // a plan-owned scratch buffer comes from hipMalloc (256-byte aligned)
  const Schedule sc = make_schedule(p, geo, g->dtype, g->data, g->scratch, T);
  out[0] = sc.apps[0];
  out[1] = sc.launches[0];
  out[2] = sc.apps[1];
  out[3] = sc.launches[1];
  if (final_copy) *final_copy = sc.final_copy ? 1 : 0;
  return STENCIL_OK;
}

int stencil_run(stencil_plan p, stencil_grid *g, int64_t T) {
  set_error("");
  Geom geo;
  if (int rc = check_run(p, g, T, geo)) return rc;
  const size_t bytes = (size_t)geo.count() * esize(g->dtype);
  if (T == 0) return STENCIL_OK;

  int device = 0;
  STENCIL_HIP_TRY(hipGetDevice(&device));
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, g->data) != hipSuccess ||
      attr.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(STENCIL_E_ARG, "data is not a device pointer");
  }
  if (int rc = ensure_operators(p, device, g->dtype)) return rc;
  DeviceState &d = p->dev[device];
  if (p->boundary == STENCIL_DIRICHLET) return run_dirichlet(p, g, T, geo, d);
  void *scratch = g->scratch;
  if (!scratch) {
    if (d.scratch_bytes < bytes) {
      if (d.scratch) {
        STENCIL_HIP_TRY(hipDeviceSynchronize());
        drop_graphs(d);
        (void)hipFree(d.scratch);
        d.scratch = nullptr;
        d.scratch_bytes = 0;
      }
      STENCIL_HIP_TRY(hipMalloc(&d.scratch, bytes));
      d.scratch_bytes = bytes;
    }
    scratch = d.scratch;
  }
  // A graph replay costs more than launching a few kernels directly (the
  // 1e6-point FP64 heat line at T = 100 is two launches: 31.8 us direct,
  // about 40 us replayed), so runs of at most kGraphMinLaunches launches are
  // launched directly even when graphs are on.
  bool direct = !p->use_graph;
  if (!direct) {
    const Schedule sc = make_schedule(p, geo, g->dtype, g->data, scratch, T);
    direct = sc.launches[0] + sc.launches[1] + (sc.final_copy ? 1 : 0) <= kGraphMinLaunches;
  }
  if (direct) return enqueue_run(p, geo, g->dtype, g->data, scratch, T, d,
                                 (hipStream_t)g->stream);
  // the run's launches captured once per (data, scratch, shape, dtype, T)
  std::ostringstream ks;
  ks << g->data << ":" << scratch << ":" << geo.nz << "x" << geo.ny << "x" << geo.nx << ":"
     << g->dtype << ":" << T;
  const std::string key = ks.str();
  auto it = d.graphs.find(key);
  if (it == d.graphs.end()) {
    if (d.graphs.size() >= kMaxRunGraphs) drop_graphs(d);
    hipStream_t cs = nullptr;
    STENCIL_HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int rc = STENCIL_OK;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      rc = enqueue_run(p, geo, g->dtype, g->data, scratch, T, d, cs);
      e = hipStreamEndCapture(cs, &graph);
    }
    if (e == hipSuccess && rc == STENCIL_OK) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (rc != STENCIL_OK || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc != STENCIL_OK ? rc : hip_fail(e, "run graph capture");
    }
    d.graph_src[key] = graph;
    it = d.graphs.emplace(key, exec).first;
  }
  STENCIL_HIP_TRY(hipGraphLaunch(it->second, (hipStream_t)g->stream));
  return STENCIL_OK;
}

int stencil_residual(const void *u, const void *ref, int dtype, int64_t n,
                     void *stream, double *out) {
  set_error("");
  if (!u || !out) return fail(STENCIL_E_ARG, "u and out must be non-NULL");
  if (dtype != STENCIL_F32 && dtype != STENCIL_F64)
    return fail(STENCIL_E_ARG, "dtype must be STENCIL_F32 or STENCIL_F64");
  if (n < 0) return fail(STENCIL_E_ARG, "n must be >= 0");
  if (n == 0) {
    out[0] = out[1] = out[2] = 0.0;
    return STENCIL_OK;
  }
  const int nblocks = 512;
  double *buf = nullptr;
  STENCIL_HIP_TRY(hipMalloc(&buf, sizeof(double) * (nblocks * 5 + 3)));
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_residual(u, ref, dtype, n, buf, nblocks, buf + nblocks * 5, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(out, buf + nblocks * 5, sizeof(double) * 3,
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (e != hipSuccess) return hip_fail(e, "stencil_residual");
  return STENCIL_OK;
}

void stencil_plan_destroy(stencil_plan p) {
  if (!p) return;
  evict_batched_plan(p);
  free_plan_devices(p);
  delete p;
}

}  // extern "C"
