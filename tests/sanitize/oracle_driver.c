/* Host sanitizer run of the oracle's C sweeps (AddressSanitizer and
 * UndefinedBehaviorSanitizer, CPU only): every entry point on small grids of
 * 1, 2 and 3 dimensions, both boundaries, a nonzero ghost value, sides
 * shorter than the stencil, T = 0, and the rejected arguments.  Checks a
 * dyadic constant field stays constant (weights 1/4, 1/2, 1/4 per axis, exact
 * in binary), so the run also means something beyond "no report". */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_num_threads(void);
int oracle_sweep_gv_f64(int, const int64_t *, int, const double *, const double *, int64_t, int,
                        double, double *);
int oracle_sweep_gv_f32(int, const int64_t *, int, const float *, const float *, int64_t, int,
                        float, float *);
int oracle_sweep_bc_f64(int, const int64_t *, int, const double *, const double *, int64_t, int,
                        double *);
int oracle_sweep_f64(int, const int64_t *, int, const double *, const double *, int64_t, double *);
int oracle_sweep_f32(int, const int64_t *, int, const float *, const float *, int64_t, float *);

static int fails = 0;
#define CHECK(c)                                              \
  do {                                                        \
    if (!(c)) {                                               \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++fails;                                                \
    }                                                         \
  } while (0)

/* dense (2r+1)^dim weights: the product of 1D (1/4, 1/2, 1/4) at r = 1, or of
 * (1/16, 1/4, 3/8, 1/4, 1/16) at r = 2 */
static void product_weights(int dim, int r, double *w) {
  const double w1[3] = {0.25, 0.5, 0.25};
  const double w2[5] = {0.0625, 0.25, 0.375, 0.25, 0.0625};
  const double *a = r == 1 ? w1 : w2;
  const int s = 2 * r + 1;
  const int n = dim == 1 ? s : dim == 2 ? s * s : s * s * s;
  for (int i = 0; i < n; ++i) {
    double v = 1.0;
    int k = i;
    for (int d = 0; d < dim; ++d) {
      v *= a[k % s];
      k /= s;
    }
    w[i] = v;
  }
}

int main(void) {
  CHECK(oracle_num_threads() >= 1);
  const int64_t shapes[][3] = {{7, 1, 1}, {1, 1, 1}, {2, 1, 1}, {5, 6, 1}, {1, 3, 1},
                               {4, 5, 6}, {2, 2, 2}, {3, 1, 4}};
  const int dims[] = {1, 1, 1, 2, 2, 3, 3, 3};
  for (int c = 0; c < 8; ++c) {
    const int dim = dims[c];
    for (int r = 1; r <= 2; ++r) {
      double w[125];
      float w32[125];
      product_weights(dim, r, w);
      const int nw = dim == 1 ? 2 * r + 1 : dim == 2 ? (2 * r + 1) * (2 * r + 1)
                                                     : (2 * r + 1) * (2 * r + 1) * (2 * r + 1);
      for (int i = 0; i < nw; ++i) w32[i] = (float)w[i];
      int64_t n = 1;
      for (int d = 0; d < dim; ++d) n *= shapes[c][d];
      double *u = malloc(sizeof(double) * (size_t)n), *v = malloc(sizeof(double) * (size_t)n);
      float *uf = malloc(sizeof(float) * (size_t)n), *vf = malloc(sizeof(float) * (size_t)n);
      for (int64_t i = 0; i < n; ++i) {
        u[i] = 0.5;
        uf[i] = 0.5f;
      }
      for (int64_t T = 0; T <= 3; ++T) {
        CHECK(oracle_sweep_f64(dim, shapes[c], r, w, u, T, v) == 0);
        for (int64_t i = 0; i < n; ++i) CHECK(v[i] == 0.5);
        CHECK(oracle_sweep_f32(dim, shapes[c], r, w32, uf, T, vf) == 0);
        for (int64_t i = 0; i < n; ++i) CHECK(vf[i] == 0.5f);
        /* ghosts equal to the field: the field stays constant */
        CHECK(oracle_sweep_gv_f64(dim, shapes[c], r, w, u, T, 1, 0.5, v) == 0);
        for (int64_t i = 0; i < n; ++i) CHECK(v[i] == 0.5);
        CHECK(oracle_sweep_gv_f32(dim, shapes[c], r, w32, uf, T, 1, 0.5f, vf) == 0);
        for (int64_t i = 0; i < n; ++i) CHECK(vf[i] == 0.5f);
        /* zero ghosts: values stay in [0, 0.5] */
        CHECK(oracle_sweep_bc_f64(dim, shapes[c], r, w, u, T, 1, v) == 0);
        for (int64_t i = 0; i < n; ++i) CHECK(v[i] >= 0.0 && v[i] <= 0.5);
      }
      /* in place (u0 and out alias) */
      CHECK(oracle_sweep_f64(dim, shapes[c], r, w, u, 2, u) == 0);
      for (int64_t i = 0; i < n; ++i) CHECK(u[i] == 0.5);
      free(u);
      free(v);
      free(uf);
      free(vf);
    }
  }
  /* rejected arguments */
  const int64_t s3[3] = {4, 4, 4};
  double w[27] = {0}, u[64] = {0}, v[64];
  CHECK(oracle_sweep_f64(0, s3, 1, w, u, 1, v) != 0);
  CHECK(oracle_sweep_f64(4, s3, 1, w, u, 1, v) != 0);
  CHECK(oracle_sweep_f64(3, s3, 1, w, u, -1, v) != 0);
  CHECK(oracle_sweep_bc_f64(3, s3, 1, w, u, 1, 2, v) != 0);
  const int64_t bad[3] = {4, 0, 4};
  CHECK(oracle_sweep_f64(3, bad, 1, w, u, 1, v) != 0);
  if (fails) {
    fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  printf("oracle sanitizer run: ok\n");
  return 0;
}
