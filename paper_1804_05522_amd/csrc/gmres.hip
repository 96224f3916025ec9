// GMRES-IR for the refinement of a HODLR solve (a production pattern, not in
// the paper): the correction equation M d = r (r = b - M x, the exact FP64
// residual) is solved by restarted GMRES in flexible form, preconditioned on
// the right by the solve with the reduced-precision factors, z_j = M_low^{-1}
// v_j, the exact product w = M z_j, classical Gram-Schmidt run twice against
// the basis, Givens rotations on the Hessenberg column, and d = Z y after m
// iterations.  Every problem of a batch runs its own GMRES in lock step: the
// basis vectors are concatenated like all vectors, and the small per-problem
// quantities (Hessenberg column, rotations, right-hand side g, y) are arrays
// indexed by problem.  Fixed m and no host decisions, so a cycle can be
// captured in a HIP graph.  Row kernels run on a grid of (2048-row slices,
// problems), like k_step_update.
#include "internal.hpp"

namespace hfde {

constexpr int kGmMax = 16;       // largest m
constexpr int kGmRows = 2048;    // rows of one row-kernel work-group (256 threads x 8)

// Per-problem small arrays of one GMRES cycle (device, problem-major).
struct GmState {
  double* H;      // batch x (kGmMax + 1) x kGmMax: H[b][i][j] at (b * (kGmMax + 1) + i) * kGmMax + j
  double* g;      // batch x (kGmMax + 1)
  double* cs;     // batch x kGmMax
  double* sn;     // batch x kGmMax
  double* h1;     // slices x batch x (kGmMax + 1): first Gram-Schmidt pass, partial sums per slice
  double* h2;     // slices x batch x (kGmMax + 1): second pass
  double* nrm;    // slices x batch: partial sums of squares
  double* y;      // batch x kGmMax
  int slices;
};

__device__ inline double gm_block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double s = red[0];
  __syncthreads();
  return s;
}

__device__ inline double gm_sum_slices(const double* part, int slices, int batch, int item, int stride, int k) {
  double s = 0.0;
  for (int q = 0; q < slices; ++q) s += part[(int64_t(q) * batch + item) * stride + k];
  return s;
}

// Partial sums of squares of v per (slice, problem): S.nrm[slice][b].
__global__ void __launch_bounds__(256) k_gm_norm2(DevPtrs P, const double* v, GmState S, int batch) {
  __shared__ double red[256];
  const Item it = P.items[blockIdx.y];
  const int64_t r0 = int64_t(blockIdx.x) * kGmRows;
  double acc = 0.0;
  for (int q = 0; q < kGmRows / 256; ++q) {
    const int64_t i = r0 + q * 256 + threadIdx.x;
    if (i < it.n) acc = fma(v[it.row0 + i], v[it.row0 + i], acc);
  }
  const double s = gm_block_sum(acc, red);
  if (threadIdx.x == 0) S.nrm[int64_t(blockIdx.x) * batch + blockIdx.y] = s;
}

// dst = src / ||src|| per problem (zero for a zero vector).  slot >= 0: the
// norm also goes to the Hessenberg matrix, H[b][slot + 1][slot] (an Arnoldi
// step's subdiagonal); slot == -1: to g[b][0], with g[b][1..] = 0 (the start of
// a cycle).
__global__ void __launch_bounds__(256) k_gm_normalize(DevPtrs P, const double* src, double* dst, GmState S, int batch,
                                                      int slot) {
  const Item it = P.items[blockIdx.y];
  double s2 = 0.0;
  for (int q = 0; q < S.slices; ++q) s2 += S.nrm[int64_t(q) * batch + blockIdx.y];
  const double nr = sqrt(fmax(s2, 0.0));
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  const int64_t r0 = int64_t(blockIdx.x) * kGmRows;
  for (int q = 0; q < kGmRows / 256; ++q) {
    const int64_t i = r0 + q * 256 + threadIdx.x;
    if (i < it.n) dst[it.row0 + i] = src[it.row0 + i] * inv;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (slot >= 0) {
      S.H[(int64_t(blockIdx.y) * (kGmMax + 1) + slot + 1) * kGmMax + slot] = nr;
    } else {
      S.g[int64_t(blockIdx.y) * (kGmMax + 1)] = nr;
      for (int k = 1; k <= kGmMax; ++k) S.g[int64_t(blockIdx.y) * (kGmMax + 1) + k] = 0.0;
    }
  }
}

// Partial inner products h[slice][b][i] = v_i^T w over the slice's rows, i <= j
// (V column-major with leading dimension ldv).
__global__ void __launch_bounds__(256) k_gm_dots(DevPtrs P, const double* V, int64_t ldv, int j, const double* w,
                                                 double* h, int batch) {
  __shared__ double red[256];
  const Item it = P.items[blockIdx.y];
  const int64_t r0 = int64_t(blockIdx.x) * kGmRows;
  double wv[kGmRows / 256];
#pragma unroll
  for (int q = 0; q < kGmRows / 256; ++q) {
    const int64_t i = r0 + q * 256 + threadIdx.x;
    wv[q] = i < it.n ? w[it.row0 + i] : 0.0;
  }
  for (int k = 0; k <= j; ++k) {
    const double* vk = V + int64_t(k) * ldv + it.row0;
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < kGmRows / 256; ++q) {
      const int64_t i = r0 + q * 256 + threadIdx.x;
      if (i < it.n) acc = fma(vk[i], wv[q], acc);
    }
    const double s = gm_block_sum(acc, red);
    if (threadIdx.x == 0) h[(int64_t(blockIdx.x) * batch + blockIdx.y) * (kGmMax + 1) + k] = s;
  }
}

// w -= sum_{i <= j} h_i v_i per problem, h summed over the slices.
__global__ void __launch_bounds__(256) k_gm_subtract(DevPtrs P, const double* V, int64_t ldv, int j, double* w,
                                                     const double* h, GmState S, int batch) {
  __shared__ double hs[kGmMax + 1];
  const Item it = P.items[blockIdx.y];
  if (threadIdx.x <= j) hs[threadIdx.x] = gm_sum_slices(h, S.slices, batch, blockIdx.y, kGmMax + 1, threadIdx.x);
  __syncthreads();
  const int64_t r0 = int64_t(blockIdx.x) * kGmRows;
  for (int q = 0; q < kGmRows / 256; ++q) {
    const int64_t i = r0 + q * 256 + threadIdx.x;
    if (i >= it.n) continue;
    double acc = w[it.row0 + i];
    for (int k = 0; k <= j; ++k) acc = fma(-hs[k], V[int64_t(k) * ldv + it.row0 + i], acc);
    w[it.row0 + i] = acc;
  }
}

// Column j of the Hessenberg matrix (the two Gram-Schmidt passes; the
// subdiagonal entry is already in H), the earlier rotations applied to it, a
// new rotation that zeroes its subdiagonal, and g rotated (one thread a problem).
__global__ void k_gm_givens(GmState S, int batch, int j) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  double col[kGmMax + 1];
  for (int k = 0; k <= j; ++k)
    col[k] = gm_sum_slices(S.h1, S.slices, batch, b, kGmMax + 1, k) + gm_sum_slices(S.h2, S.slices, batch, b, kGmMax + 1, k);
  double* Hb = S.H + int64_t(b) * (kGmMax + 1) * kGmMax;
  col[j + 1] = Hb[(j + 1) * kGmMax + j];
  for (int k = 0; k < j; ++k) {
    const double c = S.cs[b * kGmMax + k], s = S.sn[b * kGmMax + k];
    const double a = col[k], d = col[k + 1];
    col[k] = c * a + s * d;
    col[k + 1] = -s * a + c * d;
  }
  const double a = col[j], d = col[j + 1];
  const double r = hypot(a, d);
  const double c = r > 0.0 ? a / r : 1.0, s = r > 0.0 ? d / r : 0.0;
  S.cs[b * kGmMax + j] = c;
  S.sn[b * kGmMax + j] = s;
  col[j] = r;
  col[j + 1] = 0.0;
  for (int k = 0; k <= j + 1; ++k) Hb[k * kGmMax + j] = col[k];
  double* gb = S.g + int64_t(b) * (kGmMax + 1);
  const double gj = gb[j];
  gb[j] = c * gj;
  gb[j + 1] = -s * gj;
}

// y = R^{-1} g for the rotated (upper triangular) m x m Hessenberg matrix,
// one thread a problem; a zero diagonal (an exhausted Krylov space) ends the
// substitution with the remaining entries zero.
__global__ void k_gm_solve_y(GmState S, int batch, int m) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const double* Hb = S.H + int64_t(b) * (kGmMax + 1) * kGmMax;
  const double* gb = S.g + int64_t(b) * (kGmMax + 1);
  double* yb = S.y + int64_t(b) * kGmMax;
  int mm = m;
  for (int k = 0; k < m; ++k)
    if (!(fabs(Hb[k * kGmMax + k]) > 0.0)) { mm = k; break; }
  for (int k = mm; k < m; ++k) yb[k] = 0.0;
  for (int k = mm - 1; k >= 0; --k) {
    double acc = gb[k];
    for (int l = k + 1; l < mm; ++l) acc -= Hb[k * kGmMax + l] * yb[l];
    yb[k] = acc / Hb[k * kGmMax + k];
  }
}

// d = Z y per problem (Z column-major with leading dimension ldz, m columns).
__global__ void __launch_bounds__(256) k_gm_combine(DevPtrs P, const double* Z, int64_t ldz, int m, GmState S,
                                                    double* d) {
  __shared__ double ys[kGmMax];
  const Item it = P.items[blockIdx.y];
  if (threadIdx.x < m) ys[threadIdx.x] = S.y[int64_t(blockIdx.y) * kGmMax + threadIdx.x];
  __syncthreads();
  const int64_t r0 = int64_t(blockIdx.x) * kGmRows;
  for (int q = 0; q < kGmRows / 256; ++q) {
    const int64_t i = r0 + q * 256 + threadIdx.x;
    if (i >= it.n) continue;
    double acc = 0.0;
    for (int k = 0; k < m; ++k) acc = fma(ys[k], Z[int64_t(k) * ldz + it.row0 + i], acc);
    d[it.row0 + i] = acc;
  }
}

}  // namespace hfde
