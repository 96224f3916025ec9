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
//
// Finite elements (eq. (sylv-timestepping-fe)): A X E_y + E_x X B^T = C with
// the mass matrices E.  This is A~ X + X B~^T = C~ for A~ = E_x^{-1} A,
// B~ = E_y^{-1} B, C~ = E_x^{-1} C E_y^{-1}; running the recurrence above on
// it and carrying G^ = E_x G~, H^ = E_y H~ instead gives
//   Z_j = (A + q_j E_x)^{-1} G^_{j-1},  G^_j = G^_{j-1} - (p_j + q_j) E_x Z_j
// (and the same for Y, H^), with G^_J H^_J^T the residual of the generalized
// equation: no inverse of E is ever applied, the shifted operators are
// A + q_j E_x (the shift multiplies the mass matrix), and only the residual
// update gains a tridiagonal product.
#include "internal.hpp"

namespace hfde {

// E v at row i of a column of n rows (zero outside), E = mass (I + mc (S + S^T));
// mc == 0: E = I (the value itself, bit for bit).
__device__ inline double mass_at(const double* v, int64_t i, int64_t n, double mass, double mc) {
  if (mc == 0.0) return v[i];
  const double l = i > 0 ? v[i - 1] : 0.0, r = i + 1 < n ? v[i + 1] : 0.0;
  return mass * (v[i] + mc * (l + r));
}

struct MassPair {
  double mx, cx, my, cy;
};

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
  int32_t* capped;          // device bit mask: bit `mslot` set when the rank cap truncated above tau (may be null)
  double* flops;            // device accumulator of the core's algorithmic flops (may be null)
  double tau;               // absolute truncation tolerance
  double tau_rel;           // relative truncation tolerance (times ||X Y^T||_F)
  const double* tau_sq;     // if set: also tau_sq_scale * sqrt(*tau_sq) (a squared norm held on the device)
  double tau_sq_scale;
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
  double tau = fmax(jb.tau, jb.tau_rel * fro);
  if (jb.tau_sq) tau = fmax(tau, jb.tau_sq_scale * sqrt(fmax(*jb.tau_sq, 0.0)));
  RecompressOut res = wg_recompress_core(GX, GY, R, tau, jb.rmax, MU, MU + kMaxCat * kRS, Lds);
  if (threadIdx.x == 0) {
    *jb.rank_out = res.rank;
    if (res.capped && jb.capped) atomicOr(jb.capped, 1 << jb.mslot);
    if (jb.flops) {
      // work model of the core on R concatenated columns, output rank r: the
      // norm from the Grams (2 R^2), two pivoted Cholesky factorisations
      // (R^3 / 3 each), their product (2 R^3 / 3), QR with column pivoting
      // stopped after r + 1 steps (4 R^2 (r + 1)), the two transfer matrices
      // (2 R^2 r each)
      const double Rd = R, rd = res.rank;
      atomicAdd(jb.flops, 2.0 * Rd * Rd + 4.0 * Rd * Rd * Rd / 3.0 + 4.0 * Rd * Rd * (rd + 1.0) + 4.0 * Rd * Rd * rd);
    }
  }
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

// G -= w E_x Z, H -= w E_y Y for the fADI residual factors (E = I for
// differences).  Z, Y columns: r (device count).
__global__ void k_adi_update(int64_t nx, int64_t ny, const int32_t* rdev, double w, const double* Z, int64_t ldz,
                             const double* Y, int64_t ldy, double* G, int64_t ldg, double* H, int64_t ldh, MassPair E) {
  const int r = *rdev;
  const int64_t tot = (nx + ny) * r;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = e / (nx + ny), i = e % (nx + ny);
    if (i < nx) G[i + c * ldg] -= w * mass_at(Z + c * ldz, i, nx, E.mx, E.cx);
    else H[(i - nx) + c * ldh] -= w * mass_at(Y + c * ldy, i - nx, ny, E.my, E.cy);
  }
}

// The residual update of one shift pair fused with the copy that feeds the
// next pair's solves: G -= w E_x Z, H -= w E_y Y (as k_adi_update), and the
// updated columns also go to the next pair's rows of the solve workspace
// (xg, xh).  Z, Y and xg, xh are rows of different problems of the shifted
// batch, so nothing read is written.
__global__ void k_adi_update_copy(int64_t nx, int64_t ny, const int32_t* rdev, double w, const double* Z,
                                  int64_t ldz, const double* Y, int64_t ldy, double* G, int64_t ldg, double* H,
                                  int64_t ldh, double* xg, double* xh, int64_t ldxn, MassPair E) {
  const int r = *rdev;
  const int64_t tot = (nx + ny) * r;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = e / (nx + ny), i = e % (nx + ny);
    if (i < nx) {
      const double v = G[i + c * ldg] - w * mass_at(Z + c * ldz, i, nx, E.mx, E.cx);
      G[i + c * ldg] = v;
      xg[i + c * ldxn] = v;
    } else {
      const double v = H[(i - nx) + c * ldh] - w * mass_at(Y + c * ldy, i - nx, ny, E.my, E.cy);
      H[(i - nx) + c * ldh] = v;
      xh[(i - nx) + c * ldxn] = v;
    }
  }
}

// dst = scale * E src on `cols` columns of `rows` rows (E = mass (I + mc (S + S^T))).
__global__ void k_mass_cols(int64_t rows, int cols, double mass, double mc, const double* src, int64_t lds_,
                            double* dst, int64_t ldd, double scale) {
  const int64_t tot = rows * cols;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = e / rows, i = e % rows;
    dst[i + c * ldd] = scale * mass_at(src + c * lds_, i, rows, mass, mc);
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

// ---------------------------------------------------- sums of low-rank products
// S = sum_g s_g P_g Q_g^T (nx x ny) formed entry by entry in FP64: the
// residual C - A X - X B^T of a 2D step from the factors of C, of A Z_X and
// Z_X, of Z_X and B W_X.  Formed densely, its entries carry rounding errors
// of about u times the sizes of the terms, so its norm is accurate even when
// the terms cancel to 1e-10 of their size; a norm from Gram matrices of the
// concatenated factors would resolve it only to about sqrt(u).
constexpr int kLrsMax = 8;
struct LrsGroup {
  const double* P;          // nx x c, ld ldp
  int64_t ldp;
  const double* Q;          // ny x c, ld ldq
  int64_t ldq;
  const int32_t* cdev;      // c from device memory (a rank), or cfix when null
  int32_t cfix;
  double s;
};
struct LrSum {
  LrsGroup g[kLrsMax];
  int ng;
  int64_t nx, ny;
};

// 64 x 64 output tiles on the FP64 matrix cores: wave w of the four takes the
// 32 x 32 quarter (w & 1, w >> 1) as 2 x 2 tiles of 16 x 16, k-steps of four
// columns through every group.  Writes the tile's sum of squares to
// part[tile]; the entries themselves are not stored.
__global__ void __launch_bounds__(256) k_lrs_dense(const LrSum S, double* part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = int64_t(blockIdx.x) * 64 + (wave & 1) * 32;
  const int64_t c0 = int64_t(blockIdx.y) * 64 + (wave >> 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  hfde_d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = hfde_d4{0.0, 0.0, 0.0, 0.0};
  for (int gi = 0; gi < S.ng; ++gi) {
    const LrsGroup G = S.g[gi];
    const int c = G.cdev ? *G.cdev : G.cfix;
    for (int k0 = 0; k0 < c; k0 += 4) {
      const int k = k0 + lk;
      double av[2], bv[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int64_t i = r0 + 16 * t + li, j = c0 + 16 * t + li;
        av[t] = (k < c && i < S.nx) ? G.s * G.P[i + int64_t(k) * G.ldp] : 0.0;
        bv[t] = (k < c && j < S.ny) ? G.Q[j + int64_t(k) * G.ldq] : 0.0;
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[a], bv[b], acc[a][b]);
    }
  }
  double sq = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = r0 + 16 * a + 4 * v + lk, j = c0 + 16 * b + li;
        const double x = acc[a][b][v];
        if (i < S.nx && j < S.ny) sq += x * x;
      }
  __shared__ double red[256];
  red[threadIdx.x] = sq;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[int64_t(blockIdx.y) * gridDim.x + blockIdx.x] = red[0];
}

// Products of a sum S = sum_g s_g P_g Q_g^T with a thin matrix, for the
// randomized compression of S without forming it (the correction right-hand
// side of a 2D step).  side 0: Y = S Om = sum_g s_g P_g (Q_g^T Om); side 1:
// Y = S^T Om = sum_g s_g Q_g (P_g^T Om); Om has k <= kLrsK columns.  The
// inner products are formed in 32-row slices (k_lrs_cross, one slice a
// work-group, partial sums per slice), summed in slice order
// (k_lrs_cross_sum), then applied row by row (k_lrs_apply).  Every product
// has errors of about u times the sizes of the terms, as the dense form.
constexpr int kLrsK = 32;
constexpr int kLrsCols = kLrsMax * 64;   // at most 64 columns a group
constexpr int kLrsSlice = 32;

__device__ inline const double* lrs_inner(const LrsGroup& g, int side, int64_t& ld) {
  ld = side == 0 ? g.ldq : g.ldp;
  return side == 0 ? g.Q : g.P;
}

// part[slice][c][q] = sum over the slice's rows r of F[r][c] Om[r][q], F the
// concatenated inner factors (Q_g for side 0, P_g for side 1), c < total columns.
__global__ void __launch_bounds__(256) k_lrs_cross(const LrSum S, int side, const double* Om, int64_t ldo, int k,
                                                   double* part) {
  __shared__ double om[kLrsSlice][kLrsK + 1];
  __shared__ double fv[kLrsSlice][65];
  const int64_t rows = side == 0 ? S.ny : S.nx;
  const int64_t r0 = int64_t(blockIdx.x) * kLrsSlice;
  const int nr = int(min<int64_t>(kLrsSlice, rows - r0));
  for (int e = threadIdx.x; e < kLrsSlice * kLrsK; e += blockDim.x) {
    const int r = e % kLrsSlice, q = e / kLrsSlice;
    om[r][q] = (r < nr && q < k) ? Om[r0 + r + int64_t(q) * ldo] : 0.0;
  }
  int cols = 0;
  for (int gi = 0; gi < S.ng; ++gi) cols += S.g[gi].cdev ? *S.g[gi].cdev : S.g[gi].cfix;
  double* out = part + int64_t(blockIdx.x) * kLrsCols * kLrsK;
  int c0 = 0;
  for (int gi = 0; gi < S.ng; ++gi) {
    const LrsGroup G = S.g[gi];
    const int c = G.cdev ? *G.cdev : G.cfix;
    int64_t ld;
    const double* F = lrs_inner(G, side, ld);
    for (int cb = 0; cb < c; cb += 64) {
      const int cn = min(64, c - cb);
      __syncthreads();
      for (int e = threadIdx.x; e < kLrsSlice * 64; e += blockDim.x) {
        const int r = e % kLrsSlice, cc = e / kLrsSlice;
        fv[r][cc] = (r < nr && cc < cn) ? F[r0 + r + int64_t(cb + cc) * ld] : 0.0;
      }
      __syncthreads();
      for (int e = threadIdx.x; e < cn * kLrsK; e += blockDim.x) {
        const int cc = e / kLrsK, q = e % kLrsK;
        double acc = 0.0;
#pragma unroll 8
        for (int r = 0; r < kLrsSlice; ++r) acc = fma(fv[r][cc], om[r][q], acc);
        out[int64_t(c0 + cb + cc) * kLrsK + q] = acc;
      }
    }
    c0 += c;
  }
  (void)cols;
}

// T[c][q] = sum over slices of part[slice][c][q], in slice order.
__global__ void __launch_bounds__(256) k_lrs_cross_sum(const double* part, int slices, double* T) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kLrsCols * kLrsK) return;
  double acc = 0.0;
  for (int sl = 0; sl < slices; ++sl) acc += part[int64_t(sl) * kLrsCols * kLrsK + e];
  T[e] = acc;
}

// Y[i][q] = sum_g s_g sum_c O_g[i][c] T[c0_g + c][q], O the outer factors
// (P_g for side 0, Q_g for side 1), one thread a row, q < k.
__global__ void __launch_bounds__(256) k_lrs_apply(const LrSum S, int side, const double* T, int k, double* Y,
                                                   int64_t ldy) {
  const int64_t rows = side == 0 ? S.nx : S.ny;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  double acc[kLrsK];
#pragma unroll
  for (int q = 0; q < kLrsK; ++q) acc[q] = 0.0;
  int c0 = 0;
  for (int gi = 0; gi < S.ng; ++gi) {
    const LrsGroup G = S.g[gi];
    const int c = G.cdev ? *G.cdev : G.cfix;
    const double* O = side == 0 ? G.P : G.Q;
    const int64_t ld = side == 0 ? G.ldp : G.ldq;
    for (int cc = 0; cc < c; ++cc) {
      const double o = i < rows ? G.s * O[i + int64_t(cc) * ld] : 0.0;
      const double* t = T + int64_t(c0 + cc) * kLrsK;
#pragma unroll
      for (int q = 0; q < kLrsK; ++q) acc[q] = fma(o, t[q], acc[q]);
    }
    c0 += c;
  }
  if (i < rows)
    for (int q = 0; q < k; ++q) Y[i + int64_t(q) * ldy] = acc[q];
}

// out[0] = sum of the tiles' partial sums, in tile order (one work-group).
__global__ void __launch_bounds__(256) k_sum_partials(const double* part, int64_t count, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < count; e += 256) acc += part[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
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
