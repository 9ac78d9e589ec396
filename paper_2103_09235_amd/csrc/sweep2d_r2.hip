// Tiled 2D sweep, radius 2 (see sweep2d_impl.h).
#include "sweep2d_launch.h"
namespace stencil {
namespace k2d {
template hipError_t launch_r<float, 2>(const SweepLaunch &);
template hipError_t launch_r<double, 2>(const SweepLaunch &);
}  // namespace k2d
}  // namespace stencil
