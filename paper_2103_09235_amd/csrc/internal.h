// Internal declarations shared by the library's translation units.
// Not part of the public ABI (that is include/stencil.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "stencil.h"

namespace stencil {

// ----------------------------------------------------------------- errors
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

#define STENCIL_HIP_TRY(expr)                                \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return ::stencil::hip_fail(_e, #expr); \
  } while (0)

// Mask of possibly nonzero taps of an operator of radius R.
enum Mask : int {
  MASK_BOX = 0,     // all (2R+1)^d taps
  MASK_DIAMOND = 1, // |ox| + |oy| + |oz| <= R (folded star stencils)
  MASK_AXES = 2     // at most one nonzero offset coordinate (plain stars)
};

// Geometry of one grid: (nz, ny, nx) with unit leading axes for dim < 3.
struct Geom {
  int dim = 0;
  int64_t nz = 1, ny = 1, nx = 1;
  int64_t count() const { return nz * ny * nx; }
};

// One operator as the kernels consume it: weights in the grid's precision,
// dense (2R+1)^dim row-major, plus its tap list and mask.
struct OperatorDev {
  int R = 0;
  int mask = MASK_BOX;
  int ntaps = 0;             // nonzero taps
  void *w_dev = nullptr;     // dense weights on the device (T = float/double)
  void *taps_dev = nullptr;  // int4 {oz, oy, ox, widx} per nonzero tap
  std::vector<float> w32;    // host copies for by-value kernel arguments
  std::vector<double> w64;
  void *mfma_b = nullptr;    // BF16 hi/lo B-fragment table (2D FP32, R <= 8)
  bool symmetric = false;    // 2D: w[dy][dx] == w[dy][-dx] == w[-dy][dx]
  int sep_rank = 0;          // FP32: rank 1 or 2 (2D) or 1 (3D products) of a
                             // separable form cheaper than the dense taps, else 0
  std::vector<float> sep32;  // its factors: 2D a_0.., then b_0..; 3D a (z), b (y),
                             // c (x); 2R+1 each
};

// Per-device state owned by a plan.
struct DeviceState {
  OperatorDev plain32, plain64, fold32, fold64;
  bool ready32 = false, ready64 = false;
  int ready_m = 0;
  void *scratch = nullptr;
  size_t scratch_bytes = 0;
  void *dir_buf[4] = {nullptr, nullptr, nullptr, nullptr};  // zero-boundary runs:
  size_t dir_bytes = 0;      // two padded grids and two padded frame buffers
  std::map<std::string, hipGraphExec_t> graphs;
  std::map<std::string, hipGraph_t> graph_src;
};

}  // namespace stencil

struct stencil_plan_s {
  uint64_t id = 0;            // unique per plan created in this process (never reused)
  int dim = 0, r = 0, shape = 0, boundary = 0, mode = STENCIL_MODE_VECTOR;
  int max_fuse = 0;           // steps one launch may fuse; 0 = library choice
  double bvalue = 0.0;        // Dirichlet ghost value
  int use_graph = 0;          // 1 = replay periodic runs from captured hipGraphs
  const void *floor = nullptr;  // caller's floor array (device), or none
  int floor_dtype = 0;
  int64_t floor_count = 0;
  std::vector<double> w;      // plain weights, FP64, (2r+1)^dim
  int m = 1;                  // fold depth
  std::vector<double> Wm;     // folded FP64 weights, (2mr+1)^dim
  std::vector<float> Wm32;    // folded FP32 weights (rounded, compensated)
  std::vector<uint16_t> Wm_hi, Wm_lo;  // bf16 split of Wm32
  std::map<int, stencil::DeviceState> dev;
  std::map<int, std::vector<float>> batch_w32;  // folded FP32 weights by m (batched runs)
};

namespace stencil {

// Free every device resource a plan holds (all devices); the plan stays valid.
void free_plan_devices(stencil_plan_s *p);
// Drop the captured run graphs of a plan (all devices).
void drop_plan_graphs(stencil_plan_s *p);
// Free every cached batched run that names the plan (batched.hip).
void evict_batched_plan(const stencil_plan_s *p);

int side_of(int R);
int64_t count_of(int dim, int R);
int mask_for(int shape, int m);

// ---------------------------------------------------------------- folding
int fold_on_device(const std::vector<double> &w, int dim, int r, int m,
                   std::vector<double> &Wm);
void round_fold_f32(const std::vector<double> &w, const std::vector<double> &Wm,
                    int dim, int R, int m, std::vector<float> &out);
uint16_t bf16_rne(float x);
// W (S x S, row-major [dy][dx]) = sum_{j<rank} a_j b_j^T by complete-pivoting
// elimination; returns the rank (max_rank + 1 if it is larger).
int low_rank_2d(const std::vector<double> &W, int S, int max_rank, std::vector<double> &a,
                std::vector<double> &b);
// W (S x S x S) = a (x) b (x) c to 1e-12 of its largest entry: the factors.
bool product_3d(const std::vector<double> &W, int S, std::vector<double> &a,
                std::vector<double> &b, std::vector<double> &c);
// FP32 rounding of factor vectors (S each) keeping each vector's sum.
void round_factors_f32(const std::vector<double> &f, int S, std::vector<float> &out);
void profitability(const std::vector<double> &w, int dim, int r, int m,
                   int64_t *naive, int64_t *folded);

// ---------------------------------------------------------------- kernels
struct SweepLaunch {
  const void *in = nullptr;
  void *out = nullptr;
  Geom g;
  int dtype = STENCIL_F32;
  const OperatorDev *op = nullptr;
  int steps = 1;       // operator applications fused into this launch
  bool sym = false;    // mode SYMMETRIC: share mirrored partial sums if the operator allows
  bool sep = false;    // mode SEPARABLE: low-rank form if the operator has one
  const void *floor = nullptr;  // 1D: u = maxNum(u, floor) after every step
  // Dirichlet boundary on a padded grid (fused 1D and 2D kernels): after
  // every fused step the values outside rows [zbox[0], zbox[1]) x columns
  // [zbox[2], zbox[3]) (1D: columns only) are zval, the ghosts of the
  // unpadded grid.
  bool zb = false;
  int zbox[4] = {0, 0, 0, 0};
  double zval = 0.0;  // the ghost value the box's outside holds
  hipStream_t stream = nullptr;
};

// Generic kernel: one thread per point, any dim / radius, canonical order.
hipError_t launch_naive(const SweepLaunch &L);
// Device copy of n elements of esize bytes (a kernel, graph-capture safe).
hipError_t launch_copy(const void *src, void *dst, int64_t bytes, hipStream_t s);
// Tiled kernels; return hipErrorNotSupported if the case is not covered.
hipError_t launch_sweep1d(const SweepLaunch &L);
hipError_t launch_sweep2d(const SweepLaunch &L);
hipError_t launch_sweep3d(const SweepLaunch &L);
// 2D operators of radius <= 8 as BF16x3 matrix-core products (FP32 grids).
hipError_t launch_mfma2d(const SweepLaunch &L);
// Host-built B-fragment table the matrix-core kernel loads per lane.
std::vector<uint16_t> mfma_b_table(const std::vector<float> &w, int R);
// Game of Life generations on a periodic uint8 grid (life.hip).
hipError_t launch_life(const uint8_t *in, uint8_t *out, int64_t ny, int64_t nx, hipStream_t s);
// K generations per launch (K in {2, 4, 8, 16}, K <= life_max_steps).
int life_max_steps(int64_t ny, int64_t nx, const void *in, const void *out);
hipError_t launch_life_fused(const uint8_t *in, uint8_t *out, int64_t ny, int64_t nx, int K,
                             hipStream_t s);
// Largest number of fused steps the 1D kernel takes per launch.
int sweep1d_max_steps(const SweepLaunch &L);
// 2D FP32 temporal blocking: the most steps one launch fuses (1 = none), and
// the launch of 2 <= L.steps <= that many steps.
int sweep2d_max_steps(const SweepLaunch &L);
hipError_t launch_sweep2d_tb(const SweepLaunch &L);
// 3D FP32 operators of tensor rank one (op.sep_rank == 1, op.sep32 = the
// z, y and x factors): three 1D passes per point.
hipError_t launch_sweep3d_sep(const SweepLaunch &L);
// 3D FP32 temporal blocking: the most applications one launch fuses (1 =
// none), and the launch of 2 <= L.steps <= that many.
int sweep3d_max_steps(const SweepLaunch &L);
hipError_t launch_sweep3d_tb(const SweepLaunch &L);

// Zero-boundary runs (dirichlet.hip).  Padded arrays have extents np, the
// interior starting at off with extents n (z, y, x).
hipError_t dirichlet_box_copy(const void *src, int64_t sbase, int64_t ssz, int64_t ssy, void *dst,
                              int64_t dbase, int64_t dsz, int64_t dsy, const int64_t e[3],
                              int dtype, hipStream_t s);
// One plain step at the interior points closer than W to a face.
hipError_t dirichlet_frame_step(const void *src, void *dst, const int64_t np[3],
                                const int64_t off[3], const int64_t n[3], int64_t W,
                                const OperatorDev &op, int dtype, hipStream_t s);
// Set every pad point of a padded array to the ghost value.
hipError_t dirichlet_clear_pad(void *dst, const int64_t np[3], const int64_t off[3],
                               const int64_t n[3], int dtype, double value, hipStream_t s);

// FP64 fold convolution: out = a (radius Ra) * w (radius r), dim d.
hipError_t launch_fold_conv(const double *a, int Ra, const double *w, int r,
                            int dim, double *out, hipStream_t s);

// Residual reductions.
hipError_t launch_residual(const void *u, const void *ref, int dtype, int64_t n,
                           double *partials, int nblocks, double *result,
                           hipStream_t s);

}  // namespace stencil
