#include "internal.h"
namespace stencil {
hipError_t launch_sweep3d(const SweepLaunch &) { return hipErrorNotSupported; }
}
