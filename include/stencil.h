/*
 * stencil.h -- C ABI of libstencil.so: iterated constant-coefficient stencil
 * sweeps with temporal computation folding on AMD Instinct MI355X (gfx950).
 *
 * Method: Li et al., "Reducing Redundancy in Data Organization and Arithmetic
 * Calculation for Stencil Computations" (arXiv 2103.09235).
 *  - The stencil (Section 1): every point of a d-dimensional grid at time
 *    t+1 is a weighted sum of itself and its neighbours at time t; time is
 *    the outermost loop.
 *  - Temporal computation folding (Section 3.1, Section 3.3, Eq. 4-6): m
 *    consecutive steps are replaced by one application of the m-step
 *    operator whose reassigned weights W_m are the m-fold self-convolution of
 *    the stencil's weights (the paper's "folding matrix").
 *
 * Conventions used by every entry point:
 *  - Update rule (correlation form): u_{t+1}[x] = sum_o w[o] * u_t[(x+o) mod n]
 *    per axis, periodic boundaries.
 *  - Weights are a dense FP64 array of (2r+1)^dim values in row-major order,
 *    indexed [r+oz][r+oy][r+ox] (x = last axis, fastest).
 *  - Grids are contiguous row-major device arrays, x fastest, no padding;
 *    shape[] lists the axes slowest first (numpy order).
 *  - All pointers named "device" are HIP device pointers owned by the caller;
 *    the library never frees caller memory.  Work is enqueued asynchronously
 *    on the caller's HIP stream (NULL = the null stream).
 *  - Every function returns STENCIL_OK (0) or a negative status; on failure
 *    nothing has been enqueued and stencil_last_error() describes the cause.
 *    No C++ exception or abort crosses this interface.
 *  - A plan must not be changed (fold, mode) while work using it is still in
 *    flight on a stream.  Plans are not thread-safe; distinct plans are.
 */
#ifndef STENCIL_H_
#define STENCIL_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stencil_plan_s *stencil_plan; /* opaque, library-owned */

enum { STENCIL_STAR = 0, STENCIL_BOX = 1 };           /* stencil shape       */
enum { STENCIL_PERIODIC = 0, STENCIL_DIRICHLET = 1 }; /* boundary            */
enum { STENCIL_F32 = 0, STENCIL_F64 = 1 };            /* grid element type   */
enum {
  STENCIL_MODE_VECTOR = 0,      /* tiled vector kernels (default)            */
  STENCIL_MODE_EXACT_ORDER = 1, /* one thread per point, canonical order     */
  STENCIL_MODE_MFMA_BF16X3 = 2, /* 2D box folds as BF16 hi+lo MFMA products */
  STENCIL_MODE_SYMMETRIC = 3,   /* 2D operators symmetric in x and y: mirrored
                                   inputs summed once and each row's partial
                                   sum shared by two output rows (Section 3.3,
                                   Eq. 4-6); other operators run as VECTOR   */
  STENCIL_MODE_SEPARABLE = 4    /* 2D operators of rank 1 or 2 as sums of
                                   separable terms: a horizontal then a
                                   vertical 1D pass per term (the vertical and
                                   horizontal folding of Section 3.3, Eq. 4-6);
                                   3D products a (x) b (x) c as three passes;
                                   other operators run as VECTOR             */
};
enum {
  STENCIL_OK = 0,
  STENCIL_E_ARG = -1,         /* invalid argument                           */
  STENCIL_E_UNSUPPORTED = -2, /* valid but not supported by this library    */
  STENCIL_E_NOMEM = -3,       /* device or host allocation failed           */
  STENCIL_E_DEVICE = -4,      /* HIP runtime error (message in last_error)  */
  STENCIL_E_STATE = -5        /* call out of order (e.g. no plan weights)   */
};

typedef struct {
  void *data;       /* device, caller-owned; input u_0, result u_T lands here */
  void *scratch;    /* device, caller-owned, same byte size as data and not
                       overlapping it; or NULL = plan-owned cached scratch   */
  int dtype;        /* STENCIL_F32 or STENCIL_F64                             */
  int dim;          /* must equal the plan's dim                              */
  int64_t shape[3]; /* first dim entries used, slowest axis first             */
  void *stream;     /* hipStream_t or NULL                                    */
} stencil_grid;

typedef struct {
  int autotune;           /* 1 = time candidate configurations and cache the
                             winner; 0 = cached choice or the default        */
  const char *tune_cache; /* cache file path; NULL = $STENCIL_TUNE_CACHE, or
                             no file                                          */
  int use_graph;          /* 1 = capture the launches of the time loop in one
                             hipGraph and replay it                           */
  int max_m;              /* largest fold depth the tuner may choose (>= 1)   */
  int *chosen_m;          /* out, nullable: count entries, fold depth used    */
  int *passes;            /* out, nullable: count entries, the launches per run
                             that read and write grid i once each (a fused
                             pass of several applications counts one; the
                             copy back of an odd count is not included)      */
} stencil_batch_opts;

/*
 * stencil_plan_create -- validate and copy a stencil (Section 1; the Table 1
 * families are 1D/2D/3D star and box stencils).
 *   dim      1, 2 or 3.
 *   radius   r >= 1.
 *   shape    STENCIL_STAR (weights off the axes must be zero) or STENCIL_BOX.
 *   weights  host, (2r+1)^dim finite FP64 values, copied (the caller may free
 *            them on return).
 *   boundary STENCIL_PERIODIC (every axis wraps) or STENCIL_DIRICHLET (every
 *            point outside the grid holds a constant at every step: 0 unless
 *            stencil_plan_set_boundary_value sets another; the paper states
 *            no boundary, both are readings).  Folded Dirichlet runs apply
 *            W_m at points at least (m-1)r from every face, where it equals
 *            m plain fixed-ghost steps exactly, and m plain steps in the band
 *            nearer a face; see stencil_run.
 *   out      receives the plan; the plan starts unfolded (m = 1) in
 *            STENCIL_MODE_VECTOR.
 * Errors: E_ARG for a bad argument, E_UNSUPPORTED, E_NOMEM.  No device work.
 */
int stencil_plan_create(int dim, int radius, int shape, const double *weights,
                        int boundary, stencil_plan *out);

/*
 * stencil_fold_weights -- set the plan's fold depth m and form W_m, the
 * m-fold self-convolution of the weights (Section 3.3, Eq. 4-6: merged terms
 * of the m-step expansion with reassigned weights), in FP64 on the current
 * GPU.  W_m has (2mr+1)^dim entries; its sum is (sum w)^m.
 *   m            >= 1; m = 1 means the plain sweep.
 *   out_or_null  host, nullable; if given, receives W_m (FP64, row-major).
 *   out_len      host, nullable; receives (2mr+1)^dim.
 * The FP32 weights used by FP32 grids are W_m rounded to nearest (for m >= 2
 * the centre is set so that their FP64 sum is (sum w)^m to FP32 rounding);
 * see stencil_fold_weights_f32.  Synchronous (copies W_m to the host).
 * Errors: E_ARG, E_UNSUPPORTED (m too large), E_DEVICE, E_NOMEM.
 */
int stencil_fold_weights(stencil_plan p, int m, double *out_or_null,
                         int64_t *out_len);

/*
 * stencil_fold_weights_f32 -- the FP32 weights the plan's FP32 kernels use
 * for its current fold depth.  out: host, (2mr+1)^dim floats, nullable;
 * out_len: nullable.  Errors: E_ARG.  No device work.
 */
int stencil_fold_weights_f32(stencil_plan p, float *out, int64_t *out_len);

/*
 * stencil_plan_set_mode -- choose the kernel family (STENCIL_MODE_*).
 * MFMA_BF16X3 requires a 2D plan; runs with it accept FP32 grids only.
 * SYMMETRIC requires a 2D plan; it applies to operators with
 * w[dy][dx] == w[dy][-dx] == w[-dy][dx] on grids whose rows are whole
 * 16-byte vectors, and otherwise runs the VECTOR kernels.  SEPARABLE requires
 * a 2D or 3D plan; in 2D it applies to FP32 grids whose rows are whole
 * 16-byte vectors when stencil_plan_separable reports that it applies
 * (radius m*r from 2 to 8), in 3D to FP32 grids when the operator is a
 * product a (x) b (x) c (radius m*r up to 4: an x-pass, a y-pass and a
 * z-pass, 3(2mr+1) FMAs per point), with factors rounded to FP32 keeping
 * each factor's sum, and otherwise runs the VECTOR kernels.  VECTOR and EXACT_ORDER keep the canonical
 * summation order (acc = +0, one FMA per tap, row-major offsets);
 * MFMA_BF16X3, SYMMETRIC and SEPARABLE do not.
 * Errors: E_ARG, E_UNSUPPORTED.
 */
int stencil_plan_set_mode(stencil_plan p, int mode);

/*
 * stencil_plan_set_fusion -- the most operator applications one launch may
 * fuse (temporal blocking: Section 3.4 keeps several time steps of a tile on
 * chip between loads).  The 1D kernels and the 2D VECTOR kernels (FP32
 * radius 1-4, FP64 radius 1-2; radius-1 stars up to 10 steps in FP32, 14 in
 * FP64, radius-1 boxes up to 8; rows of
 * whole 16-byte vectors, at least 256 FP32 or 128 FP64 columns) fuse steps
 * in registers; the 3D FP32 VECTOR kernels (the radius-1
 * star 3 steps, the radius-1 box 2, the folded star of radius 2 two
 * applications) stream them through LDS pipeline stages.  Either way the
 * result equals one launch per application bit for bit.  0 = the library's
 * choice (default), 1 = one application per launch, k > 1 = at most k.
 * Errors: E_ARG.  No device work.
 */
int stencil_plan_set_fusion(stencil_plan p, int max_steps);

/*
 * stencil_plan_set_boundary_value -- the value every point outside the grid
 * holds at every step for a STENCIL_DIRICHLET plan (0 by default; the paper
 * states no boundary, so the boundary and its value are readings).  A tap
 * on a ghost adds weight * value in its place in the canonical chain (a zero
 * value adds nothing).  FP32 runs use the value rounded to FP32.  Folded
 * applications stay exact: a point at least (m-1)r from every face reaches
 * the ghosts only through the initial state of the m steps it replaces, and
 * the band nearer the faces takes m plain steps.
 * Errors: E_ARG (not finite), E_UNSUPPORTED (a nonzero value on a periodic
 * plan).  No device work.
 */
int stencil_plan_set_boundary_value(stencil_plan p, double value);

/*
 * stencil_plan_set_graph -- 1 = stencil_run records the launches of a
 * periodic run (the time loop of Section 1: floor(T/m) folded and T mod m
 * plain applications, plus the final copy of an odd launch count) once in a
 * hipGraph, captured on a private stream, and replays it on g->stream; the
 * graph is kept per (data, scratch, shape, dtype, T) and dropped when the
 * plan changes (fold depth, mode, fusion, floor).  Results equal the direct
 * launches bit for bit.  Zero-boundary runs, and runs of at most 4
 * launches (a replay costs more than that many direct launches), always
 * launch directly.  0 = launch directly (default).  Errors: E_ARG.  No
 * device work.
 */
int stencil_plan_set_graph(stencil_plan p, int on);

/*
 * stencil_plan_separable -- rank of the plan's current 2D operator (W_m, or
 * w when unfolded) as a matrix W[dy][dx], by Gaussian elimination with
 * complete pivoting in FP64 (pivots at most 1e-12 of the largest weight end
 * it), and whether STENCIL_MODE_SEPARABLE applies it: rank 1 or 2 and
 * 2 * rank * (2mr+1) FMAs per point fewer than its nonzero taps.  The
 * paper's unit box folds to rank 1 for every m (Section 3.3, Eq. 4); the
 * 5-point star folds to rank m+1.  3D plans: rank 1 if the operator is a
 * product a (x) b (x) c (every weight matches to 1e-12 of the largest), else
 * 0; applies if so and 3 * (2mr+1) is fewer than the nonzero taps.  rank
 * and applies are nullable; a 1D plan reports 0 and 0.  Errors: E_ARG.  No
 * device work.
 */
int stencil_plan_separable(stencil_plan p, int *rank, int *applies);

/*
 * stencil_plan_set_floor -- an obstacle applied after every step:
 * u_{t+1} = maxNum(A u_t, floor), elementwise (the American put option
 * pricing benchmark of Table 1, APOP: a 1D 3-point stencil over two arrays,
 * the option value and its exercise payoff, keeping the larger).
 *   floor  device, caller-owned, count elements of dtype, read by every run
 *          of this plan until replaced; NULL removes the floor.
 * The update is no longer linear: runs need fold depth 1 and VECTOR mode
 * (else E_UNSUPPORTED), a grid of the floor's dtype and count (else E_ARG).
 * Steps are still fused several per launch (the floor values of a lane stay
 * in registers); each step is the canonical chain followed by the max.
 * Errors: E_ARG; E_UNSUPPORTED unless the plan is 1D, radius <= 8, periodic.
 * No device work.
 */
int stencil_plan_set_floor(stencil_plan p, const void *floor, int dtype, int64_t count);

/*
 * stencil_life -- T generations of Conway's Game of Life (Table 1: a cell's
 * update depends on its 8 neighbours) on a periodic ny x nx grid of uint8
 * cells, 0 dead and 1 alive (other values are not allowed): a cell is alive
 * in the next generation iff it has exactly 3 live neighbours, or 2 and is
 * alive.  Not linear, so never folded.
 *   cells    device, caller-owned, row-major (x fastest); the result lands here.
 *   scratch  device, caller-owned, ny*nx bytes, not overlapping cells.
 *   stream   hipStream_t or NULL.  Asynchronous; T = 0 is a no-op.
 * Several generations run per launch where the grid allows (a wavefront
 * streams a strip through one pipeline stage per generation), with the same
 * result as one launch per generation.
 * Errors: E_ARG, E_UNSUPPORTED (grid too large), E_DEVICE.
 */
int stencil_life(void *cells, void *scratch, int64_t ny, int64_t nx, int64_t T, void *stream);

/*
 * stencil_life_launches -- the number of kernel launches stencil_life makes
 * for T generations on an ny x nx grid with 4-byte aligned buffers (grids
 * whose rows are whole 4-cell words, at least 256 cells wide and 33 rows
 * tall, run 16, 8, 4 or 2 generations per launch), not counting the final
 * copy an odd launch count adds.  Host only.  Errors: E_ARG.
 */
int stencil_life_launches(int64_t ny, int64_t nx, int64_t T, int64_t *launches);

/*
 * stencil_plan_info -- read back plan parameters (any pointer may be NULL):
 * dimension, radius r, fold depth m, folded radius m*r, mode.
 */
int stencil_plan_info(stencil_plan p, int *dim, int *radius, int *m,
                      int *folded_radius, int *mode);

/*
 * stencil_profitability -- scalar profitability analysis (Section 3.2,
 * Eq. 1-3) for fold depth m, by enumeration of the stencil's support S:
 *   naive  = |S| * sum_{j=0}^{m-1} |S^(+j)|  (S^(+j) = j-fold sum set,
 *            S^(+0) = {0}): one |S|-way weighted sum per distinct point of
 *            each intermediate level of the m-step expansion;
 *   folded = |S^(+m)|: one term per point of the folded stencil.
 * The profitable index is naive / folded (2D 9-point box, m = 2: 90 / 25).
 * Errors: E_ARG.  No device work.
 */
int stencil_profitability(stencil_plan p, int m, int64_t *naive,
                          int64_t *folded);

/*
 * stencil_run -- advance a grid by T original time steps (Section 1; time
 * outermost, two arrays alternating between odd and even steps as in the
 * Jacobi scheme of Section 3.3).  With fold depth m the library runs
 * floor(T/m) folded sweeps of W_m (halo width m*r) and then T mod m plain
 * sweeps; if the number of sweeps is odd a final device copy puts the result
 * back into g->data.
 *   g->dtype F32 or F64 (MFMA mode: F32 only); g->dim must equal the plan's;
 *   periodic plans need every axis >= 2*m*r + 1 (else E_UNSUPPORTED),
 *   zero-boundary plans any axis >= 1.  T = 0 is a no-op; T < 0 is E_ARG.
 *   g->scratch, when given, must not overlap g->data.
 * Dirichlet (STENCIL_DIRICHLET) runs copy the grid into plan-owned buffers
 * padded by m*r on each face, the pad holding the ghost value (four padded
 * grids, kept for later runs), run each application there and copy the
 * result back; g->scratch is not used.  Plain applications of 2D VECTOR
 * plans and of 1D plans (every mode but EXACT_ORDER) fuse several per
 * launch, the fused kernels writing the ghost value outside the grid after
 * every step; folded applications run one per launch.
 * Enqueued asynchronously on g->stream; the caller keeps data and scratch
 * alive until that work has completed.
 * Errors: E_ARG, E_UNSUPPORTED, E_STATE, E_NOMEM, E_DEVICE.
 */
int stencil_run(stencil_plan p, stencil_grid *g, int64_t T);

/*
 * stencil_run_schedule -- the launches stencil_run(p, g, T) would enqueue,
 * with no device work: out[0] applications of W_m in out[1] launches, then
 * out[2] applications of the plain weights in out[3] launches (a launch
 * fuses one or more applications; see stencil_plan_set_fusion), and
 * *final_copy (nullable) = 1 if the run ends with the device copy back into
 * g->data.  Takes the same arguments and returns the same argument errors as
 * stencil_run (the pointers are only compared, never dereferenced).
 *   out  host, 4 int64_t.
 * Errors: E_ARG, E_UNSUPPORTED.
 */
int stencil_run_schedule(stencil_plan p, const stencil_grid *g, int64_t T,
                         int64_t *out, int *final_copy);

/*
 * stencil_run_batched -- advance count independent 2D grids by T steps each
 * (Section 1's time loop per grid), grids[i] with plans[i] (plans may repeat;
 * every plan must be 2D, periodic, radius <= 2; grids FP32).  Grids that a
 * fused strip fits (at least 17 rows and 55 columns at radius 1, 119 at
 * radius 2) run their applications several per pass (up to 8 at radius 1, 4
 * at radius 2; Section 3.4's steps kept on chip), the others one persistent
 * launch per sweep over all of them together; grids whose pass count is odd
 * are copied back into data.  With opts->use_graph the whole time loop is
 * captured once in one hipGraph and replayed on grids[0].stream (all grids
 * must name the same stream).  Every grid needs a caller scratch buffer.
 * Per (stencil, radius, size class = floor(log2(side))) the library uses a
 * fold depth m <= opts->max_m, a fused-strip height, a cap on the
 * applications one fused pass takes (a lower cap narrows the border a strip
 * discards) and a strip layout (widest strips, or 128- and 64-column ones
 * only).  With opts->autotune, the classes the cache does not hold are
 * tuned together on this batch (its shapes and plans, run on scratch copies
 * of its buffers): coordinate descent from the defaults, each candidate
 * timed on the whole batch and kept only if the batch runs at least 1%
 * faster (the evaluation section leaves parameter tuning to future work).
 * Otherwise the choices come from the cache file, else the defaults (m = 1,
 * 64 rows, the kernel's cap, widest strips).  Cache lines:
 * "stencil-batched-{m,rows,kc,narrow} shape r class value".  The plans' own
 * fold depth is not changed.  Results equal the plain canonical-order sweep
 * of the chosen operators bit for bit.  opts may be NULL (no tuning, no
 * graph, m = 1).  The library keeps device tables (and the graph) of the last
 * four batches, keyed by every argument (each plan by an id that no other
 * plan of the process ever takes, not by its address); destroying a plan
 * frees the cached batches that name it.
 * Errors: E_ARG, E_UNSUPPORTED, E_NOMEM, E_DEVICE.
 */
int stencil_run_batched(const stencil_plan *plans, stencil_grid *grids,
                        int count, int64_t T, const stencil_batch_opts *opts);

/*
 * stencil_residual -- FP64 Neumaier-compensated reductions on the GPU, for the
 * mass and long-horizon residual checks:
 *   out[0] = sum_i u[i]; out[1] = sum_i |u[i] - ref[i]|;
 *   out[2] = max_i |u[i] - ref[i]|  (out[1], out[2] are 0 when ref is NULL).
 *   u, ref: device arrays of n elements of dtype; out: host, 3 doubles.
 * Synchronous on stream.  The result is deterministic (fixed reduction tree).
 * Errors: E_ARG, E_NOMEM, E_DEVICE.
 */
int stencil_residual(const void *u, const void *ref, int dtype, int64_t n,
                     void *stream, double *out);

/*
 * stencil_residual_noalloc -- the reductions of stencil_residual, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): no hipMalloc, hipFree or
 * allocating library call, no host synchronisation.
 *   u, ref, dtype, n  as for stencil_residual (ref nullable).
 *   stream            hipStream_t or NULL; the work is enqueued there.
 *   out_dev           device, caller-owned, 3 doubles: receives sum u,
 *                     sum |u - ref|, max |u - ref| when the stream reaches
 *                     the work (n = 0 gives 0, 0, 0).
 * The 512 per-block partial sums live in a fixed per-device array of the
 * library (32 KiB, held until the process ends); every call on a GPU reuses
 * that GPU's array, so calls that overlap on one GPU (other streams, other
 * threads) race and must be serialised by the caller.  The array's address
 * is looked up on the first call on each device.  The reduction tree is the
 * one stencil_residual uses, so the results are bit-identical to it.
 * Errors: E_ARG, E_UNSUPPORTED (partials larger than the array: never with
 * the library's compiled-in sizes), E_DEVICE.
 */
int stencil_residual_noalloc(const void *u, const void *ref, int dtype, int64_t n,
                             void *stream, double *out_dev);

/* stencil_plan_destroy -- free the plan and everything it owns (weights,
 * cached scratch, graphs, and the cached batched runs that name it).  NULL is
 * ignored.  The caller must ensure no work using the plan is still in
 * flight. */
void stencil_plan_destroy(stencil_plan p);

/* stencil_last_error -- thread-local description of the last failure on
 * this thread ("" if none).  Valid until the next call on this thread. */
const char *stencil_last_error(void);

/* stencil_version -- library version string. */
const char *stencil_version(void);

#ifdef __cplusplus
}
#endif

#endif /* STENCIL_H_ */
