/*
 * CPU oracle for the iterated constant-coefficient stencil sweep.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may call,
 * link or load this file; it shares no code, header or table with the HIP
 * library.  Only the tests, the smoke check and the benchmark's CPU-baseline
 * leg use it.
 *
 * What it computes is the plain definition of the method (paper, Section 1,
 * the naive (d+1)-loop stencil): time is the outermost loop and every grid
 * point at step t+1 is the weighted sum of itself and its neighbours at step
 * t.  Temporal computation folding (Section 3.1, Section 3.3, Eq. 4-6) is an
 * exact algebraic rewrite of m such steps, so the oracle of a folded run is
 * this same loop over the original steps.
 *
 * Readings that the paper leaves open (stated once here):
 *  - correlation orientation: u_{t+1}[x] = sum_o w[o] * u_t[(x + o) mod n],
 *    w stored dense with shape (2r+1)^dim, indexed [r+oz][r+oy][r+ox];
 *  - periodic boundaries in every axis, wrap(i) = ((i mod n) + n) mod n,
 *    which is defined for any n >= 1 and any |o| (multiple wraps alias, as
 *    in the circulant operator); or (the paper is silent on boundaries) zero
 *    Dirichlet ghosts: every point outside the grid holds 0 at every step,
 *    and a tap that reads one is skipped (fma(w, 0, acc) = acc for the
 *    accumulators of this chain, which start at +0 and never become -0);
 *  - canonical operation order: acc = +0.0, then one fused multiply-add per
 *    nonzero tap in row-major offset order (oz, oy, ox ascending);
 *  - two arrays alternate between odd and even steps (Section 3.3, the
 *    Jacobi two-array scheme).
 *
 * The FP64 sweep is the oracle proper.  The FP32 sweep is the same loop with
 * float and fmaf; it is the bit-exact reference for GPU kernels that keep
 * the canonical order.  Build: gcc -O2 -fopenmp -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int64_t wrap_index(int64_t i, int64_t n) { return ((i % n) + n) % n; }

/* Shape of a grid as (nz, ny, nx) with unit leading axes for dim < 3, and the
 * per-axis radius (0 on the unit axes). */
typedef struct {
  int64_t n[3];
  int rad[3];
} geom_t;

static int make_geom(int dim, const int64_t *shape, int r, geom_t *g) {
  if (dim < 1 || dim > 3 || r < 0) return -1;
  for (int a = 0; a < 3; ++a) {
    g->n[a] = 1;
    g->rad[a] = 0;
  }
  for (int a = 0; a < dim; ++a) {
    if (shape[a] < 1) return -1;
    g->n[3 - dim + a] = shape[a];
    g->rad[3 - dim + a] = r;
  }
  return 0;
}

/* Per-axis table: tab[a][i + rad] = wrap(i) for i in [-rad, n + rad), or
 * with zero ghosts (boundary 1) i itself inside the grid and -1 outside. */
static int64_t *make_wrap_table(int64_t n, int rad, int boundary) {
  int64_t len = n + 2 * (int64_t)rad;
  int64_t *t = (int64_t *)malloc(sizeof(int64_t) * (size_t)len);
  if (!t) return NULL;
  for (int64_t i = -rad; i < n + rad; ++i)
    t[i + rad] = boundary ? ((i >= 0 && i < n) ? i : -1) : wrap_index(i, n);
  return t;
}

/* Nonzero taps in row-major offset order. */
typedef struct {
  int64_t count;
  int *oz, *oy, *ox;
  int64_t *widx;
} taps_t;

static int make_taps_f64(const geom_t *g, const double *w, taps_t *t) {
  int sz = 2 * g->rad[0] + 1, sy = 2 * g->rad[1] + 1, sx = 2 * g->rad[2] + 1;
  int64_t total = (int64_t)sz * sy * sx;
  t->oz = (int *)malloc(sizeof(int) * (size_t)total);
  t->oy = (int *)malloc(sizeof(int) * (size_t)total);
  t->ox = (int *)malloc(sizeof(int) * (size_t)total);
  t->widx = (int64_t *)malloc(sizeof(int64_t) * (size_t)total);
  if (!t->oz || !t->oy || !t->ox || !t->widx) return -1;
  t->count = 0;
  for (int a = 0; a < sz; ++a)
    for (int b = 0; b < sy; ++b)
      for (int c = 0; c < sx; ++c) {
        int64_t k = ((int64_t)a * sy + b) * sx + c;
        if (w[k] != 0.0) {
          t->oz[t->count] = a - g->rad[0];
          t->oy[t->count] = b - g->rad[1];
          t->ox[t->count] = c - g->rad[2];
          t->widx[t->count] = k;
          t->count++;
        }
      }
  return 0;
}

static void free_taps(taps_t *t) {
  free(t->oz);
  free(t->oy);
  free(t->ox);
  free(t->widx);
}

/*
 * oracle_sweep_gv_f64: u_T = A^T u_0 with the canonical FMA chain, FP64.
 * dim in {1,2,3}; shape[dim] in numpy order (slowest first, x last);
 * w dense (2r+1)^dim; u0 and out hold prod(shape) values (they may alias);
 * boundary 0 = periodic, 1 = Dirichlet ghosts: every point outside the grid
 * holds the value ghost at every step.  A tap on a ghost is skipped when
 * ghost is 0 (it would add a zero product) and is an FMA with ghost, in its
 * place in the chain, otherwise.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int oracle_sweep_gv_f64(int dim, const int64_t *shape, int r, const double *w,
                        const double *u0, int64_t T, int boundary, double ghost,
                        double *out) {
  geom_t g;
  if (make_geom(dim, shape, r, &g) || T < 0 || boundary < 0 || boundary > 1) return -1;
  int64_t N = g.n[0] * g.n[1] * g.n[2];
  taps_t taps;
  double *a = (double *)malloc(sizeof(double) * (size_t)N);
  double *b = (double *)malloc(sizeof(double) * (size_t)N);
  int64_t *tz = make_wrap_table(g.n[0], g.rad[0], boundary);
  int64_t *ty = make_wrap_table(g.n[1], g.rad[1], boundary);
  int64_t *tx = make_wrap_table(g.n[2], g.rad[2], boundary);
  int rc = -1;
  if (!a || !b || !tz || !ty || !tx || make_taps_f64(&g, w, &taps)) goto done;
  memcpy(a, u0, sizeof(double) * (size_t)N);
  for (int64_t t = 0; t < T; ++t) {
    const int64_t nz = g.n[0], ny = g.n[1], nx = g.n[2];
#pragma omp parallel for collapse(3) schedule(static)
    for (int64_t z = 0; z < nz; ++z)
      for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) {
          double acc = 0.0;
          for (int64_t k = 0; k < taps.count; ++k) {
            int64_t zz = tz[z + taps.oz[k] + g.rad[0]];
            int64_t yy = ty[y + taps.oy[k] + g.rad[1]];
            int64_t xx = tx[x + taps.ox[k] + g.rad[2]];
            if (zz < 0 || yy < 0 || xx < 0) { /* ghost */
              if (ghost != 0.0) acc = fma(w[taps.widx[k]], ghost, acc);
              continue;
            }
            acc = fma(w[taps.widx[k]], a[(zz * ny + yy) * nx + xx], acc);
          }
          b[(z * ny + y) * nx + x] = acc;
        }
    double *s = a;
    a = b;
    b = s;
  }
  memcpy(out, a, sizeof(double) * (size_t)N);
  rc = 0;
  free_taps(&taps);
done:
  free(a);
  free(b);
  free(tz);
  free(ty);
  free(tx);
  return rc;
}

/*
 * oracle_sweep_gv_f32: the same definition and operation order in FP32
 * (fmaf).  Weights and the ghost value are FP32 as the kernels hold them.
 */
int oracle_sweep_gv_f32(int dim, const int64_t *shape, int r, const float *w,
                        const float *u0, int64_t T, int boundary, float ghost,
                        float *out) {
  geom_t g;
  if (make_geom(dim, shape, r, &g) || T < 0 || boundary < 0 || boundary > 1) return -1;
  int64_t N = g.n[0] * g.n[1] * g.n[2];
  int sz = 2 * g.rad[0] + 1, sy = 2 * g.rad[1] + 1, sx = 2 * g.rad[2] + 1;
  int64_t W = (int64_t)sz * sy * sx;
  double *wd = (double *)malloc(sizeof(double) * (size_t)W);
  taps_t taps;
  float *a = (float *)malloc(sizeof(float) * (size_t)N);
  float *b = (float *)malloc(sizeof(float) * (size_t)N);
  int64_t *tz = make_wrap_table(g.n[0], g.rad[0], boundary);
  int64_t *ty = make_wrap_table(g.n[1], g.rad[1], boundary);
  int64_t *tx = make_wrap_table(g.n[2], g.rad[2], boundary);
  int rc = -1;
  if (!wd || !a || !b || !tz || !ty || !tx) goto done;
  for (int64_t k = 0; k < W; ++k) wd[k] = (double)w[k];
  if (make_taps_f64(&g, wd, &taps)) goto done;
  memcpy(a, u0, sizeof(float) * (size_t)N);
  for (int64_t t = 0; t < T; ++t) {
    const int64_t nz = g.n[0], ny = g.n[1], nx = g.n[2];
#pragma omp parallel for collapse(3) schedule(static)
    for (int64_t z = 0; z < nz; ++z)
      for (int64_t y = 0; y < ny; ++y)
        for (int64_t x = 0; x < nx; ++x) {
          float acc = 0.0f;
          for (int64_t k = 0; k < taps.count; ++k) {
            int64_t zz = tz[z + taps.oz[k] + g.rad[0]];
            int64_t yy = ty[y + taps.oy[k] + g.rad[1]];
            int64_t xx = tx[x + taps.ox[k] + g.rad[2]];
            if (zz < 0 || yy < 0 || xx < 0) { /* ghost */
              if (ghost != 0.0f) acc = fmaf(w[taps.widx[k]], ghost, acc);
              continue;
            }
            acc = fmaf(w[taps.widx[k]], a[(zz * ny + yy) * nx + xx], acc);
          }
          b[(z * ny + y) * nx + x] = acc;
        }
    float *s = a;
    a = b;
    b = s;
  }
  memcpy(out, a, sizeof(float) * (size_t)N);
  rc = 0;
  free_taps(&taps);
done:
  free(wd);
  free(a);
  free(b);
  free(tz);
  free(ty);
  free(tx);
  return rc;
}

/* Periodic (boundary 0) or zero-ghost (boundary 1) sweeps. */
int oracle_sweep_bc_f64(int dim, const int64_t *shape, int r, const double *w,
                        const double *u0, int64_t T, int boundary, double *out) {
  return oracle_sweep_gv_f64(dim, shape, r, w, u0, T, boundary, 0.0, out);
}

int oracle_sweep_bc_f32(int dim, const int64_t *shape, int r, const float *w,
                        const float *u0, int64_t T, int boundary, float *out) {
  return oracle_sweep_gv_f32(dim, shape, r, w, u0, T, boundary, 0.0f, out);
}

/* The periodic sweeps (boundary 0). */
int oracle_sweep_f64(int dim, const int64_t *shape, int r, const double *w,
                     const double *u0, int64_t T, double *out) {
  return oracle_sweep_bc_f64(dim, shape, r, w, u0, T, 0, out);
}

int oracle_sweep_f32(int dim, const int64_t *shape, int r, const float *w,
                     const float *u0, int64_t T, float *out) {
  return oracle_sweep_bc_f32(dim, shape, r, w, u0, T, 0, out);
}
