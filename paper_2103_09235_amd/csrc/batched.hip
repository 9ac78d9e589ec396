#include "internal.h"
extern "C" int stencil_run_batched(const stencil_plan *plans, stencil_grid *grids,
                                   int count, int64_t T,
                                   const stencil_batch_opts *) {
  stencil::set_error("");
  if (count < 0 || T < 0) return stencil::fail(STENCIL_E_ARG, "count and T must be >= 0");
  if (count == 0 || T == 0) return STENCIL_OK;
  if (!plans || !grids) return stencil::fail(STENCIL_E_ARG, "plans and grids must be non-NULL");
  for (int i = 0; i < count; ++i)
    if (!plans[i] || !grids[i].data) return stencil::fail(STENCIL_E_ARG, "NULL plan or data");
  return stencil::fail(STENCIL_E_UNSUPPORTED, "batched runs are not available yet");
}
