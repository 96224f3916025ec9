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

constexpr int kLrRows = 1024;
constexpr int kLrSub = 32;

__global__ void __launch_bounds__(256) k_lr_gram(const LrJob* jobs, const LrUnit* units, double* partial) {
  __shared__ double xs[kLrSub * kMaxCat];
  const LrUnit u = units[blockIdx.x];
  const LrJob jb = jobs[u.job];
  const Cat3V A = resolve(u.which == 0 ? jb.X : jb.Y);
  const int64_t rows = u.which == 0 ? jb.rows_x : jb.rows_y;
  const int M = A.cols();
  const int t = threadIdx.x;
  const int ti = (t % 16) * 4, tj = (t / 16) * 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  const int64_t r0 = int64_t(u.chunk) * kLrRows, r1 = min<int64_t>(rows, r0 + kLrRows);
  for (int64_t s0 = r0; s0 < r1; s0 += kLrSub) {
    const int sr = int(min<int64_t>(kLrSub, r1 - s0));
    __syncthreads();
    for (int e = t; e < kLrSub * kMaxCat; e += 256) {
      const int i = e % kLrSub, c = e / kLrSub;
      xs[e] = (i < sr && c < M) ? A.at(s0 + i, c) : 0.0;
    }
    __syncthreads();
    if (ti < M && tj < M) {
      for (int i = 0; i < sr; ++i) {
        double xv[4], yv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) xv[a] = xs[i + (ti + a) * kLrSub];
#pragma unroll
        for (int b = 0; b < 4; ++b) yv[b] = xs[i + (tj + b) * kLrSub];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] += xv[a] * yv[b];
      }
    }
  }
  double* out = partial + int64_t(u.out) * kG2;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) out[(ti + a) + (tj + b) * kMaxCat] = acc[a][b];
}

__global__ void __launch_bounds__(kWG) k_lr_core(const LrJob* jobs, const double* G, double* Mbuf) {
  extern __shared__ double Lds[];
  const LrJob jb = jobs[blockIdx.x];
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
__global__ void __launch_bounds__(256) k_lr_form(const LrJob* jobs, const LrUnit* units, const double* Mbuf) {
  __shared__ double Ms[kMaxCat * kRS];
  const LrUnit u = units[blockIdx.x];
  const LrJob jb = jobs[u.job];
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
__global__ void k_lr_frob(const LrJob* jobs, const double* G, double* out) {
  __shared__ double red[256];
  const LrJob jb = jobs[blockIdx.x];
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
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
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

}  // namespace hfde
