#include "internal.h"
namespace stencil {
hipError_t launch_sweep1d(const SweepLaunch &) { return hipErrorNotSupported; }
int sweep1d_max_steps(const SweepLaunch &) { return 1; }
}
