// Dispatch of the tiled 2D sweep (sweep2d_impl.h) over element type and
// radius; the instantiations live in sweep2d_r*.hip.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace stencil {
namespace k2d {
template <typename T, int R>
hipError_t launch_r(const SweepLaunch &L);
}  // namespace k2d

hipError_t launch_sweep2d(const SweepLaunch &L) {
  using k2d::launch_r;
  if (L.steps != 1) return hipErrorNotSupported;
  if (L.g.ny > (1 << 30) || L.g.nx > (1 << 30) || L.g.nx * L.g.ny > (1LL << 40))
    return hipErrorNotSupported;
  const int R = L.op->R;
  if (L.dtype == STENCIL_F32) {
    switch (R) {
      case 1: return launch_r<float, 1>(L);
      case 2: return launch_r<float, 2>(L);
      case 3: return launch_r<float, 3>(L);
      case 4: return launch_r<float, 4>(L);
      case 5: return launch_r<float, 5>(L);
      case 6: return launch_r<float, 6>(L);
      case 7: return launch_r<float, 7>(L);
      case 8: return launch_r<float, 8>(L);
      default: return hipErrorNotSupported;
    }
  }
  switch (R) {
    case 1: return launch_r<double, 1>(L);
    case 2: return launch_r<double, 2>(L);
    case 3: return launch_r<double, 3>(L);
    case 4: return launch_r<double, 4>(L);
    default: return hipErrorNotSupported;
  }
}

}  // namespace stencil
