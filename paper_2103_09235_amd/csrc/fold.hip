// Temporal computation folding: the m-step operator's weights.
//
// Folding m steps merges the repeated terms of the m-step expansion of a
// point and reassigns their weights (Section 3.1; the folding matrix of
// Section 3.3, Eq. 4-6).  For a constant-coefficient stencil the reassigned
// weights are exactly the m-fold self-convolution W_m = w * w * ... * w:
// applying w twice gives sum_a w[a] sum_b w[b] u[x+a+b] =
// sum_o (sum_{a+b=o} w[a] w[b]) u[x+o].  W_m is formed here in FP64 on the
// GPU by m-1 convolutions with w; the FP32 and BF16 forms are derived on the
// host from it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <set>

#include "internal.h"

namespace stencil {

int side_of(int R) { return 2 * R + 1; }

int64_t count_of(int dim, int R) {
  int64_t s = side_of(R), c = 1;
  for (int i = 0; i < dim; ++i) c *= s;
  return c;
}

int mask_for(int shape, int m) {
  if (shape == STENCIL_BOX) return MASK_BOX;
  return m == 1 ? MASK_AXES : MASK_DIAMOND;
}

// out[o] = sum_b w[b] * a[o - b], o in [-(Ra+r), Ra+r]^d, b in [-r, r]^d in
// row-major order, one FMA per term that lands inside a's support.
__global__ void k_fold_conv(const double *__restrict__ a, int Ra,
                            const double *__restrict__ w, int r, int dim,
                            double *__restrict__ out) {
  const int Ro = Ra + r, so = 2 * Ro + 1, sa = 2 * Ra + 1, sw = 2 * r + 1;
  int64_t total = 1;
  for (int i = 0; i < dim; ++i) total *= so;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < total;
       p += (int64_t)gridDim.x * blockDim.x) {
    int o[3] = {0, 0, 0};
    int64_t q = p;
    for (int i = dim - 1; i >= 0; --i) {
      o[i] = (int)(q % so) - Ro;
      q /= so;
    }
    double acc = 0.0;
    int64_t nb = 1;
    for (int i = 0; i < dim; ++i) nb *= sw;
    for (int64_t bi = 0; bi < nb; ++bi) {
      int b[3] = {0, 0, 0};
      int64_t t = bi;
      for (int i = dim - 1; i >= 0; --i) {
        b[i] = (int)(t % sw) - r;
        t /= sw;
      }
      bool inside = true;
      int64_t ai = 0;
      for (int i = 0; i < dim; ++i) {
        int d = o[i] - b[i];
        if (d < -Ra || d > Ra) inside = false;
        ai = ai * sa + (d + Ra);
      }
      if (inside) acc = fma(w[bi], a[ai], acc);
    }
    out[p] = acc;
  }
}

hipError_t launch_fold_conv(const double *a, int Ra, const double *w, int r,
                            int dim, double *out, hipStream_t s) {
  int64_t total = count_of(dim, Ra + r);
  int threads = 256;
  int blocks = (int)std::min<int64_t>((total + threads - 1) / threads, 1024);
  hipLaunchKernelGGL(k_fold_conv, dim3(blocks), dim3(threads), 0, s, a, Ra, w,
                     r, dim, out);
  return hipGetLastError();
}

int fold_on_device(const std::vector<double> &w, int dim, int r, int m,
                   std::vector<double> &Wm) {
  if (m == 1) {
    Wm = w;
    return STENCIL_OK;
  }
  const int64_t nmax = count_of(dim, m * r);
  double *d_w = nullptr, *d_a = nullptr, *d_b = nullptr;
  hipError_t e = hipMalloc(&d_w, sizeof(double) * w.size());
  if (e == hipSuccess) e = hipMalloc(&d_a, sizeof(double) * nmax);
  if (e == hipSuccess) e = hipMalloc(&d_b, sizeof(double) * nmax);
  if (e == hipSuccess)
    e = hipMemcpy(d_w, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(d_a, w.data(), sizeof(double) * w.size(), hipMemcpyHostToDevice);
  for (int k = 1; k < m && e == hipSuccess; ++k) {
    e = launch_fold_conv(d_a, k * r, d_w, r, dim, d_b, nullptr);
    std::swap(d_a, d_b);
  }
  if (e == hipSuccess) {
    Wm.assign(nmax, 0.0);
    e = hipMemcpy(Wm.data(), d_a, sizeof(double) * nmax, hipMemcpyDeviceToHost);
  }
  if (d_w) (void)hipFree(d_w);
  if (d_a) (void)hipFree(d_a);
  if (d_b) (void)hipFree(d_b);
  if (e != hipSuccess) return hip_fail(e, "fold_on_device");
  return STENCIL_OK;
}

// FP32 weights of the folded operator: nearest-even rounding of each FP64
// weight; for m >= 2 the centre weight is reset to
// fl32((sum w)^m - sum_{o != centre} fl32(W_m[o])) (both sums sequential in
// row-major order, the power by repeated multiplication), so the FP32
// operator keeps the folded operator's total weight and the mean of the
// field does not drift over many folded sweeps.  A centre that rounds to
// zero is kept as is.
void round_fold_f32(const std::vector<double> &w, const std::vector<double> &Wm,
                    int dim, int R, int m, std::vector<float> &out) {
  out.resize(Wm.size());
  for (size_t i = 0; i < Wm.size(); ++i) out[i] = (float)Wm[i];
  if (m < 2) return;
  const int64_t side = side_of(R);
  int64_t c = 0;
  for (int i = 0; i < dim; ++i) c = c * side + R;
  if (out[c] == 0.0f) return;
  double s1 = 0.0;
  for (double v : w) s1 += v;
  double target = 1.0;
  for (int k = 0; k < m; ++k) target *= s1;
  double rest = 0.0;
  for (int64_t i = 0; i < (int64_t)out.size(); ++i)
    if (i != c) rest += (double)out[i];
  out[c] = (float)(target - rest);
}

// Low-rank form of a 2D operator (the algebra behind the paper's vertical
// then horizontal folding, Section 3.3 Eq. 4-6: the folded unit box is the
// outer product of two 1D folded weight vectors): W = sum_{j<rank} a_j b_j^T
// by Gaussian elimination with complete pivoting on the S x S matrix
// W[dy][dx].  Each step takes the largest remaining entry p at (i, k) and
// removes the rank-one term col_k(E) row_i(E) / p; it stops when the largest
// remaining entry is at most 1e-12 of the largest weight (or after
// max_rank + 1 terms, reported as rank max_rank + 1).  The factors are
// balanced: a_j = col / sqrt|p|, b_j = row * sign(p) / sqrt|p|.
int low_rank_2d(const std::vector<double> &W, int S, int max_rank, std::vector<double> &a,
                std::vector<double> &b) {
  std::vector<double> E = W;
  double scale = 0.0;
  for (double v : E) scale = std::max(scale, std::fabs(v));
  a.clear();
  b.clear();
  if (scale == 0.0) return 0;
  int rank = 0;
  while (rank <= max_rank) {
    int pi = 0, pk = 0;
    double best = -1.0;
    for (int i = 0; i < S; ++i)
      for (int k = 0; k < S; ++k)
        if (std::fabs(E[i * S + k]) > best) {
          best = std::fabs(E[i * S + k]);
          pi = i;
          pk = k;
        }
    if (best <= 1e-12 * scale) break;
    const double p = E[pi * S + pk];
    const double sq = std::sqrt(std::fabs(p));
    std::vector<double> col(S), row(S);
    for (int i = 0; i < S; ++i) col[i] = E[i * S + pk];
    for (int k = 0; k < S; ++k) row[k] = E[pi * S + k];
    for (int i = 0; i < S; ++i)
      for (int k = 0; k < S; ++k) E[i * S + k] -= col[i] * row[k] / p;
    for (int i = 0; i < S; ++i) a.push_back(col[i] / sq);
    for (int k = 0; k < S; ++k) b.push_back(row[k] / (p < 0 ? -sq : sq));
    ++rank;
  }
  return rank;
}

// W (S x S x S, row-major [dz][dy][dx]) = a (x) b (x) c: the line of W
// through its largest entry along each axis gives the factor up to scale
// (for a product, W[:, y*, x*] / p, W[z*, :, x*] / p and W[z*, y*, :] / p
// with p = W[z*, y*, x*] are the normalised factors and W = p a b c); the
// scale is split evenly (cube root of p) so the three factors have equal
// size.  Returns false unless every entry matches to 1e-12 of the largest.
bool product_3d(const std::vector<double> &W, int S, std::vector<double> &a,
                std::vector<double> &b, std::vector<double> &c) {
  if ((int)W.size() != S * S * S) return false;
  int best = 0;
  for (int i = 1; i < S * S * S; ++i)
    if (std::fabs(W[i]) > std::fabs(W[best])) best = i;
  const double p = W[best];
  if (p == 0.0) return false;
  const int zs = best / (S * S), ys = (best / S) % S, xs = best % S;
  const double g = std::cbrt(p);
  a.assign(S, 0.0);
  b.assign(S, 0.0);
  c.assign(S, 0.0);
  for (int i = 0; i < S; ++i) {
    a[i] = W[(i * S + ys) * S + xs] / p * g;
    b[i] = W[(zs * S + i) * S + xs] / p * g;
    c[i] = W[(zs * S + ys) * S + i] / p * g;
  }
  const double tol = 1e-12 * std::fabs(p);
  for (int z = 0; z < S; ++z)
    for (int y = 0; y < S; ++y)
      for (int x = 0; x < S; ++x)
        if (std::fabs(W[(z * S + y) * S + x] - a[z] * b[y] * c[x]) > tol) return false;
  return true;
}

// FP32 factors with each vector's total kept: entries rounded to nearest,
// then the centre entry set to fl32(sum64 - sum of the other rounded
// entries), so the FP32 operator's total weight sum_j (sum a_j)(sum b_j)
// stays that of W (the mean of the field does not drift).
void round_factors_f32(const std::vector<double> &f, int S, std::vector<float> &out) {
  const int n = (int)f.size() / S;
  out.resize(f.size());
  for (int j = 0; j < n; ++j) {
    double total = 0.0, rest = 0.0;
    for (int i = 0; i < S; ++i) {
      total += f[j * S + i];
      out[j * S + i] = (float)f[j * S + i];
    }
    const int c = S / 2;
    if (out[j * S + c] == 0.0f) continue;
    for (int i = 0; i < S; ++i)
      if (i != c) rest += (double)out[j * S + i];
    out[j * S + c] = (float)(total - rest);
  }
}

uint16_t bf16_rne(float x) {
  uint32_t b;
  std::memcpy(&b, &x, 4);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

// Scalar profitability analysis (Section 3.2, Eq. 1-3) by enumerating the
// support S of the stencil and its sum sets S^(+j).
void profitability(const std::vector<double> &w, int dim, int r, int m,
                   int64_t *naive, int64_t *folded) {
  using P = std::array<int, 3>;
  std::set<P> S;
  const int s = 2 * r + 1;
  for (int64_t i = 0; i < (int64_t)w.size(); ++i) {
    if (w[i] == 0.0) continue;
    P p{0, 0, 0};
    int64_t t = i;
    for (int a = dim - 1; a >= 0; --a) {
      p[a] = (int)(t % s) - r;
      t /= s;
    }
    S.insert(p);
  }
  std::set<P> level{P{0, 0, 0}};
  int64_t nv = 0;
  for (int k = 0; k < m; ++k) {
    nv += (int64_t)S.size() * (int64_t)level.size();
    std::set<P> next;
    for (const P &a : level)
      for (const P &b : S) next.insert(P{a[0] + b[0], a[1] + b[1], a[2] + b[2]});
    level.swap(next);
  }
  if (naive) *naive = nv;
  if (folded) *folded = (int64_t)level.size();
}

}  // namespace stencil
