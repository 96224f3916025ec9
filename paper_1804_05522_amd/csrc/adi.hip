// 2D per-step Sylvester equation A X + X B^T = C (Sec. 4.2, eq. (sylv-timestepping))
// by factored ADI with shifted HODLR solves, on gfx950.
//
// A = 1/2 I + nu_x (D1+ T + D1- T^T), B = 1/2 I + nu_y (D2+ T + D2- T^T);
// C = U_m + dt F is kept in low-rank form C = G H^T (Sec. 4.1: sums of
// low-rank terms are recompressed by QR-type factorisations and a small core
// decomposition).  With shift pairs (p_j, q_j), p_j in the spectral interval
// of A and q_j in that of B:
//   Z_j = (A + q_j I)^{-1} G_{j-1},   Y_j = (B + p_j I)^{-1} H_{j-1},
//   X_j = X_{j-1} + (p_j + q_j) Z_j Y_j^T,
//   G_j = G_{j-1} - (p_j + q_j) Z_j,  H_j = H_{j-1} - (p_j + q_j) Y_j,
// and the residual is exactly C - A X_J - X_J B^T = G_J H_J^T (expand
// A Z_j = G_{j-1} - q_j Z_j and B Y_j = H_{j-1} - p_j Y_j).  The shifts solve
// the Zolotarev problem for the two real intervals (elliptic functions,
// host FP64); the shifted factors A + q_j I, B + p_j I are one batched HODLR
// operator whose problems share the off-diagonal blocks and differ on the
// leaf diagonals.  X is recompressed after every step (rank <= 64).
#include "internal.hpp"

namespace hfde {

// Up to three column groups, counts optionally read from device memory.
struct Grp {
  const double* p;
  int64_t ld;
  const int32_t* cnt_dev;   // if non-null, the column count is *cnt_dev
  int32_t cnt;
  double s;
};
struct Cat3 {
  Grp g[3];
  __device__ inline int count(int k) const { return g[k].cnt_dev ? *g[k].cnt_dev : g[k].cnt; }
};
struct Cat3V {          // resolved on the device
  const double* p[3];
  int64_t ld[3];
  int c[3];
  double s[3];
  __device__ inline int cols() const { return c[0] + c[1] + c[2]; }
  __device__ inline const double* colp(int col, double& scale) const {
    const int g = col < c[0] ? 0 : (col < c[0] + c[1] ? 1 : 2);
    const int cc = col - (g > 0 ? c[0] : 0) - (g > 1 ? c[1] : 0);
    const double* base = g == 0 ? p[0] : (g == 1 ? p[1] : p[2]);
    const int64_t l = g == 0 ? ld[0] : (g == 1 ? ld[1] : ld[2]);
    scale = g == 0 ? s[0] : (g == 1 ? s[1] : s[2]);
    return base + int64_t(cc) * l;
  }
  __device__ inline double at(int64_t row, int col) const {
    if (col < c[0]) return s[0] * p[0][row + int64_t(col) * ld[0]];
    col -= c[0];
    if (col < c[1]) return s[1] * p[1][row + int64_t(col) * ld[1]];
    col -= c[1];
    return s[2] * p[2][row + int64_t(col) * ld[2]];
  }
};
__device__ inline Cat3V resolve(const Cat3& a) {
  Cat3V v;
  for (int k = 0; k < 3; ++k) {
    v.p[k] = a.g[k].p;
    v.ld[k] = a.g[k].ld;
    v.c[k] = a.g[k].p ? a.count(k) : 0;
    v.s[k] = a.g[k].s;
  }
  return v;
}

// One low-rank job: X^T Y Grams / recompression of X Y^T / forms.
struct LrJob {
  Cat3 X, Y;
  int64_t rows_x, rows_y;
  int32_t gx, gy;           // Gram slots (64 x 64) for X^T X and Y^T Y
  int32_t mslot;            // transfer matrices slot (2 x 64 x 32)
  int32_t* rank_out;        // device rank of the result
  double tau;               // absolute truncation tolerance
  double tau_rel;           // relative truncation tolerance (times ||X Y^T||_F)
  int32_t rmax;
  double* U; int64_t ldu;   // form outputs
  double* V; int64_t ldv;
};

struct LrUnit {
  int32_t job;
  int32_t which;            // 0: X side, 1: Y side
  int32_t chunk;
  int32_t out;              // partial slot
};

constexpr int kLrRows = 256;     // rows per Gram partial (one work-group on the matrix cores)

// The job descriptor travels as a kernel argument; the unit lists depend only
// on the job slot and the row counts and stay resident between calls.
__global__ void __launch_bounds__(256) k_lr_gram(const LrJob jb, const LrUnit* units, double* partial) {
  __shared__ __align__(16) double st[kMaxCat * kStLd];
  const LrUnit u = units[blockIdx.x];
  const Cat3V A = resolve(u.which == 0 ? jb.X : jb.Y);
  const int64_t rows = u.which == 0 ? jb.rows_x : jb.rows_y;
  const int64_t r0 = int64_t(u.chunk) * kLrRows;
  const int64_t cnt = max<int64_t>(0, min<int64_t>(rows, r0 + kLrRows) - r0);
  // symmetric Gram A^T A of the chunk on the FP64 matrix cores (64 x 64, zero padded)
  wg_gram_mfma<false>(A, A, r0, cnt, cnt, true, partial + int64_t(u.out) * kG2, nullptr, kMaxCat, true, st, st);
}

__global__ void __launch_bounds__(kCoreWG) k_lr_core(const LrJob jb, const double* G, double* Mbuf) {
  extern __shared__ __align__(16) double Lds[];
  const Cat3V X = resolve(jb.X);
  const int R = X.cols();
  double* MU = Mbuf + int64_t(jb.mslot) * 2 * kMaxCat * kRS;
  const double* GX = G + int64_t(jb.gx) * kG2;
  const double* GY = G + int64_t(jb.gy) * kG2;
  // ||X Y^T||_F^2 = trace(G_X G_Y) (both symmetric)
  __shared__ double red[kWG];
  double s = 0.0;
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) s += GX[(e % R) + (e / R) * kMaxCat] * GY[(e % R) + (e / R) * kMaxCat];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  const double fro = sqrt(fmax(red[0], 0.0));
  __syncthreads();
  const double tau = fmax(jb.tau, jb.tau_rel * fro);
  RecompressOut res = wg_recompress_core(GX, GY, R, tau, jb.rmax, MU, MU + kMaxCat * kRS, Lds);
  if (threadIdx.x == 0) *jb.rank_out = res.rank;
}

// U = X * M_U, V = Y * M_V (row-parallel); units: (job, side, chunk of 256 rows)
__global__ void __launch_bounds__(256) k_lr_form(const LrJob jb, const LrUnit* units, const double* Mbuf) {
  __shared__ double Ms[kMaxCat * kRS];
  const LrUnit u = units[blockIdx.x];
  const Cat3V A = resolve(u.which == 0 ? jb.X : jb.Y);
  const int R = A.cols();
  const int r = *jb.rank_out;
  const double* M = Mbuf + int64_t(jb.mslot) * 2 * kMaxCat * kRS + (u.which ? kMaxCat * kRS : 0);
  g2l(M, kMaxCat, Ms, kMaxCat, R, r);
  __syncthreads();
  const int64_t rows = u.which == 0 ? jb.rows_x : jb.rows_y;
  const int64_t i = int64_t(u.chunk) * 256 + threadIdx.x;
  if (i >= rows) return;
  double* Y = u.which == 0 ? jb.U : jb.V;
  const int64_t ld = u.which == 0 ? jb.ldu : jb.ldv;
  double a[kMaxCat];
#pragma unroll
  for (int k = 0; k < kMaxCat; ++k) a[k] = k < R ? A.at(i, k) : 0.0;
  for (int c = 0; c < r; ++c) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxCat; ++k) s += a[k] * Ms[k + c * kMaxCat];
    Y[i + int64_t(c) * ld] = s;
  }
}

// ||X Y^T||_F^2 = trace((X^T X)(Y^T Y)) from the two Grams; out[slot] = value.
__global__ void k_lr_frob(const LrJob jb, const double* G, double* out) {
  __shared__ double red[256];
  const Cat3V X = resolve(jb.X);
  const int R = X.cols();
  const double* GX = G + int64_t(jb.gx) * kG2;
  const double* GY = G + int64_t(jb.gy) * kG2;
  double s = 0.0;
  for (int e = threadIdx.x; e < R * R; e += 256) s += GX[(e % R) + (e / R) * kMaxCat] * GY[(e / R) + (e % R) * kMaxCat];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// G -= w Z, H -= w Y for the fADI residual factors; also stores w Z into the
// accumulation buffer (X update operand).  Z, Y columns: r (device count).
__global__ void k_adi_update(int64_t nx, int64_t ny, const int32_t* rdev, double w, const double* Z, int64_t ldz,
                             const double* Y, int64_t ldy, double* G, int64_t ldg, double* H, int64_t ldh) {
  const int r = *rdev;
  const int64_t tot = (nx + ny) * r;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = e / (nx + ny), i = e % (nx + ny);
    if (i < nx) G[i + c * ldg] -= w * Z[i + c * ldz];
    else H[(i - nx) + c * ldh] -= w * Y[(i - nx) + c * ldy];
  }
}

// copy r (device count) columns between strided blocks, with scale
__global__ void k_copy_cols(int64_t rows, const int32_t* rdev, int rfix, const double* src, int64_t lds_, double* dst,
                            int64_t ldd, double s) {
  const int r = rdev ? *rdev : rfix;
  const int64_t tot = rows * r;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = e / rows, i = e % rows;
    dst[i + c * ldd] = s * src[i + c * lds_];
  }
}

// ---------------------------------------------------- dense fields
// Uniform(-1, 1) numbers from a counter-based generator (splitmix64 of
// seed + index), for the random sketch of a dense field.
__global__ void k_fill_uniform(double* out, int64_t count, uint64_t seed) {
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count; e += int64_t(gridDim.x) * blockDim.x) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull * uint64_t(e + 1);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    out[e] = double(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
}

__global__ void k_set_identity(double* out, int n, int ld) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * n) out[(e % n) + (e / n) * ld] = (e % n == e / n) ? 1.0 : 0.0;
}

// Y = X Om: X dense nx x ny (FP32, column-major), Om ny x k (ld ny), Y nx x k
// (ld nx), k <= 32.  A thread per row of X; Om is staged in LDS in tiles.
__global__ void __launch_bounds__(256) k_field_times(int64_t nx, int64_t ny, const float* X, const double* Om, int k,
                                                     double* Y) {
  constexpr int kT = 64;
  __shared__ double om[kT * 32];
  const int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x;
  double acc[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) acc[c] = 0.0;
  for (int64_t j0 = 0; j0 < ny; j0 += kT) {
    __syncthreads();
    for (int e = threadIdx.x; e < kT * 32; e += 256) {
      const int jj = e % kT, c = e / kT;
      om[jj * 32 + c] = (j0 + jj < ny && c < k) ? Om[j0 + jj + int64_t(c) * ny] : 0.0;
    }
    __syncthreads();
    if (i < nx) {
      const int jn = int(min<int64_t>(kT, ny - j0));
      for (int jj = 0; jj < jn; ++jj) {
        const double x = double(X[i + (j0 + jj) * nx]);
#pragma unroll
        for (int c = 0; c < 32; ++c) acc[c] += x * om[jj * 32 + c];
      }
    }
  }
  if (i < nx)
    for (int c = 0; c < k; ++c) Y[i + int64_t(c) * nx] = acc[c];
}

// B = X^T Q: X nx x ny (FP32), Q nx x k (ld nx, k = *kdev <= 32), B ny x k
// (ld ny).  A block takes 256 columns of X; 32-row tiles of X are staged
// (coalesced down the columns) and transposed in LDS with Q's rows.
__global__ void __launch_bounds__(256) k_field_t_times(int64_t nx, int64_t ny, const float* X, const double* Q,
                                                       const int32_t* kdev, double* B) {
  constexpr int kR = 32;
  __shared__ float xt[kR * 257];
  __shared__ double qs[kR * 32];
  const int k = *kdev;
  const int64_t j0 = int64_t(blockIdx.x) * 256;
  const int t = threadIdx.x;
  double acc[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) acc[c] = 0.0;
  for (int64_t i0 = 0; i0 < nx; i0 += kR) {
    __syncthreads();
    for (int e = t; e < kR * 256; e += 256) {
      const int r = e % kR, cl = e / kR;
      const int64_t i = i0 + r, j = j0 + cl;
      xt[r * 257 + cl] = (i < nx && j < ny) ? X[i + j * nx] : 0.0f;
    }
    for (int e = t; e < kR * 32; e += 256) {
      const int r = e % kR, c = e / kR;
      qs[r * 32 + c] = (i0 + r < nx && c < k) ? Q[i0 + r + int64_t(c) * nx] : 0.0;
    }
    __syncthreads();
    for (int r = 0; r < kR; ++r) {
      const double x = double(xt[r * 257 + t]);
#pragma unroll
      for (int c = 0; c < 32; ++c) acc[c] += x * qs[r * 32 + c];
    }
  }
  const int64_t j = j0 + t;
  if (j < ny)
    for (int c = 0; c < k; ++c) B[j + int64_t(c) * ny] = acc[c];
}

}  // namespace hfde
