// Host sanitizer run of the library's C ABI (AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code, CPU only): the calls that do
// no device work -- plan creation and its validation, the plan settings,
// launch schedules of every dimension, mode and boundary, the profitability
// count, the Game of Life launch count, and the error paths -- with the
// return codes the header documents.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "stencil.h"

static int fails = 0;
#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                                       \
    }                                                                \
  } while (0)

static stencil_grid grid(int dim, int64_t a, int64_t b, int64_t c, int dtype) {
  stencil_grid g{};
  g.data = reinterpret_cast<void *>(uintptr_t(1) << 30);
  g.scratch = reinterpret_cast<void *>(uintptr_t(1) << 40);
  g.dtype = dtype;
  g.dim = dim;
  g.shape[0] = a;
  g.shape[1] = b;
  g.shape[2] = c;
  return g;
}

int main() {
  // plans: valid and rejected
  std::vector<double> star2(9, 0.0), box2(9, 1.0 / 9), box3(27, 1.0 / 27), heat = {0.25, 0.5, 0.25};
  star2[1] = star2[3] = star2[5] = star2[7] = 0.1;
  star2[4] = 0.6;
  stencil_plan p2 = nullptr, b2 = nullptr, b3 = nullptr, h1 = nullptr, bad = nullptr;
  CHECK(stencil_plan_create(2, 1, STENCIL_STAR, star2.data(), STENCIL_PERIODIC, &p2) == STENCIL_OK);
  CHECK(stencil_plan_create(2, 1, STENCIL_BOX, box2.data(), STENCIL_PERIODIC, &b2) == STENCIL_OK);
  CHECK(stencil_plan_create(3, 1, STENCIL_BOX, box3.data(), STENCIL_DIRICHLET, &b3) == STENCIL_OK);
  CHECK(stencil_plan_create(1, 1, STENCIL_STAR, heat.data(), STENCIL_PERIODIC, &h1) == STENCIL_OK);
  CHECK(stencil_plan_create(0, 1, STENCIL_BOX, box2.data(), 0, &bad) == STENCIL_E_ARG);
  CHECK(stencil_plan_create(4, 1, STENCIL_BOX, box2.data(), 0, &bad) == STENCIL_E_ARG);
  CHECK(stencil_plan_create(2, 0, STENCIL_BOX, box2.data(), 0, &bad) == STENCIL_E_ARG);
  CHECK(stencil_plan_create(2, 1, 9, box2.data(), 0, &bad) == STENCIL_E_ARG);
  CHECK(stencil_plan_create(2, 1, STENCIL_STAR, box2.data(), 0, &bad) == STENCIL_E_ARG);
  CHECK(stencil_plan_create(2, 1, STENCIL_BOX, nullptr, 0, &bad) == STENCIL_E_ARG);
  std::vector<double> nan9(9, 0.0);
  nan9[4] = std::nan("");
  CHECK(stencil_plan_create(2, 1, STENCIL_BOX, nan9.data(), 0, &bad) == STENCIL_E_ARG);
  CHECK(bad == nullptr);
  CHECK(stencil_last_error()[0] != '\0');

  // settings
  CHECK(stencil_plan_set_mode(p2, STENCIL_MODE_SYMMETRIC) == STENCIL_OK);
  CHECK(stencil_plan_set_mode(p2, 99) == STENCIL_E_ARG);
  CHECK(stencil_plan_set_mode(h1, STENCIL_MODE_MFMA_BF16X3) != STENCIL_OK);
  CHECK(stencil_plan_set_mode(p2, STENCIL_MODE_VECTOR) == STENCIL_OK);
  CHECK(stencil_plan_set_fusion(p2, 3) == STENCIL_OK);
  CHECK(stencil_plan_set_fusion(p2, -1) == STENCIL_E_ARG);
  CHECK(stencil_plan_set_fusion(p2, 0) == STENCIL_OK);
  CHECK(stencil_plan_set_graph(p2, 1) == STENCIL_OK);
  CHECK(stencil_plan_set_graph(p2, 0) == STENCIL_OK);
  CHECK(stencil_plan_set_boundary_value(b3, 0.5) == STENCIL_OK);
  CHECK(stencil_plan_set_boundary_value(p2, 0.5) == STENCIL_E_UNSUPPORTED);
  CHECK(stencil_plan_set_boundary_value(b3, std::nan("")) == STENCIL_E_ARG);
  CHECK(stencil_plan_set_floor(h1, nullptr, STENCIL_F64, 0) == STENCIL_OK);
  int dim = 0, rad = 0, m = 0, R = 0, mode = 0;
  CHECK(stencil_plan_info(b3, &dim, &rad, &m, &R, &mode) == STENCIL_OK);
  CHECK(dim == 3 && rad == 1 && m == 1 && R == 1 && mode == STENCIL_MODE_VECTOR);
  int rank = -1, applies = -1;
  CHECK(stencil_plan_separable(b2, &rank, &applies) == STENCIL_OK);
  CHECK(rank == 1);
  int64_t len = 0;
  std::vector<float> w32(9);
  CHECK(stencil_fold_weights_f32(b2, w32.data(), &len) == STENCIL_OK && len == 9);

  // profitability (Section 3.2): the 9-point box at m = 2 gives 90 / 25
  int64_t naive = 0, folded = 0;
  CHECK(stencil_profitability(b2, 2, &naive, &folded) == STENCIL_OK);
  CHECK(naive == 90 && folded == 25);
  CHECK(stencil_profitability(b2, 0, &naive, &folded) == STENCIL_E_ARG);

  // launch schedules (host only; the pointers are only compared)
  int64_t out[4] = {0, 0, 0, 0};
  int copy = -1;
  stencil_grid g = grid(2, 8192, 8192, 0, STENCIL_F32);
  CHECK(stencil_run_schedule(p2, &g, 1000, out, &copy) == STENCIL_OK);
  CHECK(out[2] == 1000 && out[3] == 100 && copy == 0);
  g = grid(2, 8192, 8192, 0, STENCIL_F64);
  CHECK(stencil_run_schedule(p2, &g, 12, out, &copy) == STENCIL_OK && out[3] == 2);
  g = grid(2, 2, 8192, 0, STENCIL_F32);
  CHECK(stencil_run_schedule(p2, &g, 4, out, &copy) == STENCIL_E_UNSUPPORTED);
  g = grid(2, 64, 64, 0, STENCIL_F32);
  CHECK(stencil_run_schedule(p2, &g, -1, out, &copy) == STENCIL_E_ARG);
  CHECK(stencil_run_schedule(p2, &g, 5, nullptr, &copy) == STENCIL_E_ARG);
  g.scratch = g.data;
  CHECK(stencil_run_schedule(p2, &g, 5, out, &copy) == STENCIL_E_ARG);
  g = grid(3, 64, 64, 64, STENCIL_F32);
  CHECK(stencil_run_schedule(b3, &g, 5, out, &copy) == STENCIL_OK && copy == 1);
  g = grid(1, 1000000, 0, 0, STENCIL_F64);
  CHECK(stencil_run_schedule(h1, &g, 100, out, &copy) == STENCIL_OK && out[3] == 2);
  g = grid(3, 64, 64, 64, STENCIL_F32);
  CHECK(stencil_run_schedule(p2, &g, 5, out, &copy) == STENCIL_E_ARG);  // dim mismatch
  for (int64_t T : {0, 1, 2, 7, 37}) {
    g = grid(2, 300, 1024, 0, STENCIL_F32);
    CHECK(stencil_run_schedule(b2, &g, T, out, &copy) == STENCIL_OK);
    CHECK(out[2] == T && out[3] <= T);
  }

  // Game of Life launch counts
  int64_t launches = 0;
  CHECK(stencil_life_launches(5000, 5000, 1000, &launches) == STENCIL_OK && launches > 0);
  CHECK(stencil_life_launches(0, 5000, 10, &launches) == STENCIL_E_ARG);

  // residual argument errors (no device work)
  double res[3];
  CHECK(stencil_residual(nullptr, nullptr, STENCIL_F32, 4, nullptr, res) == STENCIL_E_ARG);
  CHECK(stencil_residual_noalloc(nullptr, nullptr, STENCIL_F32, 4, nullptr, nullptr) ==
        STENCIL_E_ARG);

  stencil_plan_destroy(p2);
  stencil_plan_destroy(b2);
  stencil_plan_destroy(b3);
  stencil_plan_destroy(h1);
  stencil_plan_destroy(nullptr);
  if (fails) {
    std::fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  std::printf("C ABI sanitizer run: ok (%s)\n", stencil_version());
  return 0;
}
