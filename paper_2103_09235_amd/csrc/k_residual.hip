// FP64 compensated reductions for the mass and residual checks of long
// runs: sum u, sum |u - ref| (Neumaier's improved Kahan-Babuska summation)
// and max |u - ref|.  The reduction tree is fixed (grid size, block size,
// pairing order), so results are bit-reproducible run to run.
#include <hip/hip_runtime.h>

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
