// FP64 compensated reductions for the mass and residual checks of long
// runs: sum u, sum |u - ref| (Neumaier's improved Kahan-Babuska summation)
// and max |u - ref|.  The reduction tree is fixed (grid size, block size,
// pairing order), so results are bit-reproducible run to run.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#include "internal.h"

namespace stencil {

namespace {

struct Acc {
  double s, c;  // running sum and its accumulated rounding error
};

__device__ __forceinline__ void neumaier_add(Acc &a, double x) {
  const double t = a.s + x;
  if (fabs(a.s) >= fabs(x))
    a.c += (a.s - t) + x;
  else
    a.c += (x - t) + a.s;
  a.s = t;
}

__device__ __forceinline__ Acc combine(Acc a, Acc b) {
  Acc r = a;
  neumaier_add(r, b.s);
  r.c += b.c;
  return r;
}

constexpr int kThreads = 256;

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_residual_partial(const T *__restrict__ u, const T *__restrict__ ref, int64_t n,
                   double *__restrict__ partials) {
  Acc su{0.0, 0.0}, sd{0.0, 0.0};
  double mx = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n; i += stride) {
    const double v = (double)u[i];
    neumaier_add(su, v);
    if (ref) {
      const double d = fabs(v - (double)ref[i]);
      neumaier_add(sd, d);
      mx = fmax(mx, d);
    }
  }
  __shared__ double sh[5][kThreads];
  sh[0][threadIdx.x] = su.s;
  sh[1][threadIdx.x] = su.c;
  sh[2][threadIdx.x] = sd.s;
  sh[3][threadIdx.x] = sd.c;
  sh[4][threadIdx.x] = mx;
  __syncthreads();
  for (int half = kThreads / 2; half > 0; half >>= 1) {
    if ((int)threadIdx.x < half) {
      const int j = threadIdx.x + half;
      Acc a = combine(Acc{sh[0][threadIdx.x], sh[1][threadIdx.x]}, Acc{sh[0][j], sh[1][j]});
      Acc b = combine(Acc{sh[2][threadIdx.x], sh[3][threadIdx.x]}, Acc{sh[2][j], sh[3][j]});
      sh[0][threadIdx.x] = a.s;
      sh[1][threadIdx.x] = a.c;
      sh[2][threadIdx.x] = b.s;
      sh[3][threadIdx.x] = b.c;
      sh[4][threadIdx.x] = fmax(sh[4][threadIdx.x], sh[4][j]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 5; ++k) partials[blockIdx.x * 5 + k] = sh[k][0];
}

__global__ void __launch_bounds__(kThreads)
k_residual_final(const double *__restrict__ partials, int nblocks,
                 double *__restrict__ result) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Acc su{0.0, 0.0}, sd{0.0, 0.0};
  double mx = 0.0;
  for (int b = 0; b < nblocks; ++b) {
    su = combine(su, Acc{partials[b * 5 + 0], partials[b * 5 + 1]});
    sd = combine(sd, Acc{partials[b * 5 + 2], partials[b * 5 + 3]});
    mx = fmax(mx, partials[b * 5 + 4]);
  }
  result[0] = su.s + su.c;
  result[1] = sd.s + sd.c;
  result[2] = mx;
}

}  // namespace

hipError_t launch_residual(const void *u, const void *ref, int dtype, int64_t n,
                           double *partials, int nblocks, double *result,
                           hipStream_t s) {
  if (dtype == STENCIL_F32)
    hipLaunchKernelGGL(k_residual_partial<float>, dim3(nblocks), dim3(kThreads), 0,
                       s, (const float *)u, (const float *)ref, n, partials);
  else
    hipLaunchKernelGGL(k_residual_partial<double>, dim3(nblocks), dim3(kThreads), 0,
                       s, (const double *)u, (const double *)ref, n, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(kThreads), 0, s, partials,
                     nblocks, result);
  return hipGetLastError();
}

}  // namespace stencil

// ------------------------------------------------ allocation-free variant
//
// The partial sums of stencil_residual_noalloc live in a fixed device array
// instead of a per-call allocation.  Host code never passes the array's name
// to a kernel (on the host it is only a stand-in for the symbol): its device
// address is looked up once per device with hipGetSymbolAddress and that
// address is what the kernels receive.
namespace {

constexpr int kResidualBlocks = 512;   // same reduction tree as stencil_residual
constexpr size_t kScratchDoubles = 4096;  // 32 KiB per device
constexpr size_t kScratchNeed = (size_t)kResidualBlocks * 5;  // per-block partials
static_assert(kScratchNeed <= kScratchDoubles, "residual partials exceed the scratch array");

static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_ptr;  // device ordinal -> address of scratch

// The device address of scratch on the current device (looked up on the
// first call there).
int scratch_on_current_device(double **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return stencil::hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return STENCIL_OK;
  }
  double *ptr = nullptr;
  e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return stencil::hip_fail(e, "hipGetSymbolAddress(scratch)");
  if (!ptr) return stencil::fail(STENCIL_E_DEVICE, "no device address for the residual scratch array");
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return STENCIL_OK;
}

}  // namespace

extern "C" int stencil_residual_noalloc(const void *u, const void *ref, int dtype, int64_t n,
                                        void *stream, double *out_dev) {
  using namespace stencil;
  set_error("");
  if (!u || !out_dev) return fail(STENCIL_E_ARG, "u and out_dev must be non-NULL");
  if (dtype != STENCIL_F32 && dtype != STENCIL_F64)
    return fail(STENCIL_E_ARG, "dtype must be STENCIL_F32 or STENCIL_F64");
  if (n < 0) return fail(STENCIL_E_ARG, "n must be >= 0");
  if (kScratchNeed > kScratchDoubles)
    return fail(STENCIL_E_UNSUPPORTED, "residual partials (" + std::to_string(kScratchNeed) +
                                           " doubles) exceed the scratch array (" +
                                           std::to_string(kScratchDoubles) + ")");
  double *ptr = nullptr;
  int rc = scratch_on_current_device(&ptr);
  if (rc != STENCIL_OK) return rc;
  // n = 0 still runs the kernels: every block writes its partials (zeros),
  // so out_dev receives 0, 0, 0 without a memset
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = launch_residual(u, ref, dtype, n, ptr, kResidualBlocks, out_dev, s);
  if (e != hipSuccess) return hip_fail(e, "stencil_residual_noalloc");
  return STENCIL_OK;
}
