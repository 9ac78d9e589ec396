#include "internal.h"
namespace stencil {
hipError_t launch_sweep2d(const SweepLaunch &) { return hipErrorNotSupported; }
}
