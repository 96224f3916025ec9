// HODLR LU factorisation (Sec. 3.5) on gfx950: one work-group per problem
// walks its tree in post-order.
//
// Block LU of a node with children c1, c2 and the Schur complement S of the
// node (the node's block of M minus the low-rank update P Q^T inherited
// from its ancestors):
//   S = [S11 S12; S21 S22],  S11 = L1 U1 (recursively, leaf LUs pivoted),
//   S12 = U12 V12^T - P1 Q2^T  -> recompressed  U12' V12'^T
//   S21 = U21 V21^T - P2 Q1^T  -> recompressed  U21' V21'^T
//   U-factor block  L1^{-1} S12 = U~12 V12'^T,   U~12 = L1^{-1} U12'
//   L-factor block  S21 U1^{-1} = U21' V~21^T,   V~21 = U1^{-T} V21'
//   S22 - S21 S11^{-1} S12 = A22 - [P2, U21' C][Q2, V12']^T,  C = V~21^T U~12
// and the pending update of c2 is recompressed before descending.  Because
// the triangular factors keep the quasiseparable rank (Sec. 3.2), the
// inverses of L and U are HODLR with the same ranks:
//   (L^{-1})21 = -(L2^{-1} U21') (L1^{-T} V~21)^T
//   (U^{-1})12 = -(U1^{-1} U~12) (U2^{-T} V12')^T
// They are formed as soon as a node is complete; the triangular solves
// inside the factorisation (L1^{-1}X, U1^{-T}X, ...) are then HODLR
// matrix products with the finished subtrees' inverse factors, and the
// per-step solve is two HODLR products.
//
// Recompression of A B^T (A: m x R, B: n x R, R <= 64): column pairs are
// balanced, Gram matrices A^T A, B^T B give triangular factors R_A, R_B by
// pivoted Cholesky, the core K = R_A R_B^T is truncated by Householder QR with
// column pivoting at the absolute tolerance tau on the Frobenius norm of the
// dropped part, and the new factors are formed without inverting R_A, R_B:
//   U' = A (R_B^T Pi R11^{-1}),  V' = B (R_A^T Q_K).
#include "internal.hpp"

namespace hfde {

// ----------------------------------------------------------------- LDS map
namespace lds {
constexpr int G = 0;                       // 64 x 65
constexpr int LA = G + kMaxCat * kLdG;     // 64 x 65
constexpr int LB = LA + kMaxCat * kLdG;
constexpr int KC = LB + kMaxCat * kLdG;
constexpr int RED = KC + kMaxCat * kLdG;   // 2048 reduction scratch
constexpr int VEC = RED + 2048;            // 512 small vectors
constexpr int IVEC = VEC + 512;            // 256 ints (128 doubles)
constexpr int TOTAL = IVEC + 128;          // doubles
// leaf phase overlays
constexpr int S = 0;
constexpr int LI = S + kMaxLeaf * kLdsLeaf;
constexpr int UI = LI + kMaxLeaf * kLdsLeaf;
constexpr int PL = UI + kMaxLeaf * kLdsLeaf;   // 64 x 32
constexpr int QL = PL + kMaxLeaf * kRS;
static_assert(QL + kMaxLeaf * kRS <= RED, "leaf overlay");
}  // namespace lds
constexpr size_t kFactorLdsBytes = size_t(lds::TOTAL) * sizeof(double);

// A column-concatenation [s1*A1, s2*A2] of two global column-major blocks.
struct Cat {
  const double* p1;
  int64_t ld1;
  int c1;
  double s1;
  const double* p2;
  int64_t ld2;
  int c2;
  double s2;
  __device__ inline double at(int64_t row, int col) const {
    return col < c1 ? s1 * p1[row + int64_t(col) * ld1] : s2 * p2[row + int64_t(col - c1) * ld2];
  }
  __device__ inline int cols() const { return c1 + c2; }
  // base of column col (its row 0) and the column's scale
  __device__ inline const double* colp(int col, double& scale) const {
    const bool first = col < c1;
    scale = first ? s1 : s2;
    return first ? p1 + int64_t(col) * ld1 : p2 + int64_t(col - c1) * ld2;
  }
};

__device__ inline Cat cat1(const double* p, int64_t ld, int c) {
  return Cat{p, ld, c, 1.0, p, ld, 0, 0.0};
}

// Copies a rows x cols column-major block from global memory (ld lsrc) into
// LDS (ld ldst), keeping `kBatch` loads in flight per thread: the loads of a
// batch are issued before any of its LDS stores, so a thread waits for one
// memory round trip per batch instead of one per element.
constexpr int kBatch = 8;
__device__ inline void g2l(const double* src, int64_t lsrc, double* dst, int ldst, int rows, int cols) {
  const int tot = rows * cols, nt = blockDim.x;
  for (int e0 = threadIdx.x; e0 < tot; e0 += nt * kBatch) {
    double v[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int e = e0 + q * nt;
      v[q] = e < tot ? src[(e % rows) + int64_t(e / rows) * lsrc] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int e = e0 + q * nt;
      if (e < tot) dst[(e % rows) + (e / rows) * ldst] = v[q];
    }
  }
}

// As g2l, and zero-fills the rest of the rows_pad x cols_pad destination, so
// that unrolled loops can run over the padded size without guards.
__device__ inline void g2l_pad(const double* src, int64_t lsrc, double* dst, int ldst, int rows, int cols,
                               int rows_pad, int cols_pad) {
  const int tot = rows_pad * cols_pad, nt = blockDim.x;
  for (int e0 = threadIdx.x; e0 < tot; e0 += nt * kBatch) {
    double v[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int e = e0 + q * nt, i = e % rows_pad, c = e / rows_pad;
      v[q] = (e < tot && i < rows && c < cols) ? src[i + int64_t(c) * lsrc] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const int e = e0 + q * nt;
      if (e < tot) dst[(e % rows_pad) + (e / rows_pad) * ldst] = v[q];
    }
  }
}

// LDS views.  A generic pointer into the work-group's LDS is converted once;
// indexing through the view is then 32-bit, and loads at constant strides
// from one base take immediate offsets (pairs of them in one instruction).
typedef __attribute__((address_space(3))) double ldsd;
typedef __attribute__((address_space(3))) int ldsi;
__device__ inline ldsd* lds_view(double* p) { return (ldsd*)p; }
__device__ inline const ldsd* lds_view(const double* p) { return (const ldsd*)p; }
__device__ inline ldsi* lds_view(int* p) { return (ldsi*)p; }

// sum_{q = lo}^{hi - 1} A[q SA] B[q SB] over LDS operands (constant strides):
// full batches of eight loads of each operand are issued before their fused
// products go into four partial sums (q mod 4), combined at the end in a
// fixed order; the last partial batch reads up to seven entries past hi
// (inside the work-group's LDS) and discards their products.
template <int SA, int SB>
__device__ inline double lds_dot(const ldsd* A, const ldsd* B, int lo, int hi) {
  double s4[4] = {0.0, 0.0, 0.0, 0.0};
  int q0 = lo;
  for (; q0 + 8 <= hi; q0 += 8) {
    const ldsd* a = A + q0 * SA;
    const ldsd* b = B + q0 * SB;
    double x[8], y[8];
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      x[w] = a[w * SA];
      y[w] = b[w * SB];
    }
#pragma unroll
    for (int w = 0; w < 8; ++w) s4[w & 3] = fma(x[w], y[w], s4[w & 3]);
  }
  if (q0 < hi) {
    const ldsd* a = A + q0 * SA;
    const ldsd* b = B + q0 * SB;
    double x[8], y[8];
#pragma unroll
    for (int w = 0; w < 8; ++w) {
      x[w] = a[w * SA];
      y[w] = b[w * SB];
    }
#pragma unroll
    for (int w = 0; w < 8; ++w) s4[w & 3] = (q0 + w < hi) ? fma(x[w], y[w], s4[w & 3]) : s4[w & 3];
  }
  return (s4[0] + s4[1]) + (s4[2] + s4[3]);
}
template <int SA, int SB>
__device__ inline double lds_dot(const double* A, const double* B, int lo, int hi) {
  return lds_dot<SA, SB>(lds_view(A), lds_view(B), lo, hi);
}

__device__ inline void wg_sync() {
  __threadfence_block();
  __syncthreads();
}

// C (LDS, ldc) = A^T B, A: K x M, B: K x N (global).  2x2 register tiles,
// K split across threads when there are fewer tiles than threads; partial
// tiles are summed in a fixed order (deterministic).
__device__ void wg_atb(const Cat& A, const Cat& B, int64_t K, double* C, int ldc, double* red) {
  const int M = A.cols(), N = B.cols();
  const int tm = (M + 1) / 2, tn = (N + 1) / 2, tiles = tm * tn;
  const int t = threadIdx.x;
  if (tiles == 0) return;
  if (tiles >= kWG / 2) {
    for (int tile = t; tile < tiles; tile += kWG) {
      const int i0 = 2 * (tile % tm), j0 = 2 * (tile / tm);
      const int i1 = i0 + 1 < M ? i0 + 1 : i0, j1 = j0 + 1 < N ? j0 + 1 : j0;
      double c00 = 0, c01 = 0, c10 = 0, c11 = 0;
      for (int64_t k = 0; k < K; ++k) {
        double a0 = A.at(k, i0), a1 = A.at(k, i1), b0 = B.at(k, j0), b1 = B.at(k, j1);
        c00 += a0 * b0; c01 += a0 * b1; c10 += a1 * b0; c11 += a1 * b1;
      }
      C[i0 + j0 * ldc] = c00;
      if (j0 + 1 < N) C[i0 + (j0 + 1) * ldc] = c01;
      if (i0 + 1 < M) C[i0 + 1 + j0 * ldc] = c10;
      if (i0 + 1 < M && j0 + 1 < N) C[i0 + 1 + (j0 + 1) * ldc] = c11;
    }
    wg_sync();
    return;
  }
  int nsplit = kWG / tiles;
  if (int64_t(nsplit) > K) nsplit = K > 0 ? int(K) : 1;
  const int tile = t % tiles, sp = t / tiles;
  if (sp < nsplit) {
    const int i0 = 2 * (tile % tm), j0 = 2 * (tile / tm);
    const int i1 = i0 + 1 < M ? i0 + 1 : i0, j1 = j0 + 1 < N ? j0 + 1 : j0;
    const int64_t k0 = K * sp / nsplit, k1 = K * (sp + 1) / nsplit;
    double c00 = 0, c01 = 0, c10 = 0, c11 = 0;
    for (int64_t k = k0; k < k1; ++k) {
      double a0 = A.at(k, i0), a1 = A.at(k, i1), b0 = B.at(k, j0), b1 = B.at(k, j1);
      c00 += a0 * b0; c01 += a0 * b1; c10 += a1 * b0; c11 += a1 * b1;
    }
    double* r = red + 4 * (sp * tiles + tile);
    r[0] = c00; r[1] = c01; r[2] = c10; r[3] = c11;
  }
  wg_sync();
  for (int e = t; e < tiles * 4; e += kWG) {
    const int tile2 = e / 4, q = e % 4;
    double s = 0;
    for (int p = 0; p < nsplit; ++p) s += red[4 * (p * tiles + tile2) + q];
    const int i = 2 * (tile2 % tm) + (q >> 1), j = 2 * (tile2 / tm) + (q & 1);
    if (i < M && j < N) C[i + j * ldc] = s;
  }
  wg_sync();
}

// Y[0:m, 0:nc] = alpha * A[0:m, :] * Msm (Msm in LDS, K x nc, ld ldm).
__device__ void wg_a_times_small(const Cat& A, int64_t m, const double* Msm, int ldm, int nc,
                                 double* Y, int64_t ldy, double alpha) {
  const int K = A.cols();
  for (int64_t e = threadIdx.x; e < m * nc; e += kWG) {
    const int64_t i = e % m;
    const int c = int(e / m);
    double s = 0;
    for (int k = 0; k < K; ++k) s += A.at(i, k) * Msm[k + c * ldm];
    Y[i + c * ldy] = alpha * s;
  }
  wg_sync();
}

__device__ void wg_copy_cols(const double* X, int64_t ldx, int64_t m, int nc, double* Y, int64_t ldy,
                             double alpha) {
  for (int64_t e = threadIdx.x; e < m * nc; e += kWG) {
    const int64_t i = e % m;
    const int c = int(e / m);
    Y[i + c * ldy] = alpha * X[i + c * ldx];
  }
  wg_sync();
}

// Wave-level reductions (wave64).
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ inline void wave_argmax(double& v, int& idx) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double ov = __shfl_xor(v, o);
    const int oi = __shfl_xor(idx, o);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

// Pivot searches inside one wave: lane-wise maximum of a 32-bit key, returned to every lane (DPP butterflies
// inside each row of 16 lanes, then the four row maxima by readlane).
__device__ inline unsigned wave_max_u32(unsigned v) {
  v = max(v, unsigned(__builtin_amdgcn_update_dpp(0, int(v), 0xB1, 0xF, 0xF, false)));   // quad_perm 1,0,3,2
  v = max(v, unsigned(__builtin_amdgcn_update_dpp(0, int(v), 0x4E, 0xF, 0xF, false)));   // quad_perm 2,3,0,1
  v = max(v, unsigned(__builtin_amdgcn_update_dpp(0, int(v), 0x141, 0xF, 0xF, false)));  // row_half_mirror
  v = max(v, unsigned(__builtin_amdgcn_update_dpp(0, int(v), 0x140, 0xF, 0xF, false)));  // row_mirror
  const unsigned a = unsigned(__builtin_amdgcn_readlane(int(v), 0)), b = unsigned(__builtin_amdgcn_readlane(int(v), 16));
  const unsigned c = unsigned(__builtin_amdgcn_readlane(int(v), 32)), d = unsigned(__builtin_amdgcn_readlane(int(v), 48));
  return max(max(a, b), max(c, d));
}

// Orders LDS accesses of one wave against each other (lanes exchange data
// through LDS inside the wave, without a work-group barrier).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ inline double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ inline double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
// Sum over the 64 lanes of a wave, in a fixed order, returned to every lane.
__device__ inline double wave_sum_fixed(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}
// Pivot key of a non-negative value: its leading 26 bits, ties to the lowest
// lane; NaN ranks first, lanes that do not take part rank last.
__device__ inline unsigned pivot_key(double a, bool part, int lane) {
  if (!part) return 0u;
  const unsigned hi = (a == a) ? unsigned(__double2hiint(a)) : 0xFFFFFFFFu;
  return (max(hi, 0x40u) & ~0x3Fu) | unsigned(63 - lane);
}
__device__ inline int pivot_lane(unsigned key) { return 63 - int(wave_max_u32(key) & 63u); }

// Pivoted Cholesky of the R x R PSD matrix G (LDS, ld kLdG), by one wave:
// G ~ Lc Lc^T with Lc (LDS, R x k, ld kLdG) in original row order.  Lane i
// owns row i; each step takes the largest remaining diagonal entry and forms
// the new column left-looking from the columns already made.  Stops when the
// largest remaining diagonal entry falls below delta * (largest initial one).
// G is read only.
__device__ int wave_pchol(const double* Gg, int R, double* Lg, double delta) {
  const ldsd* G = lds_view(Gg);
  ldsd* Lc = lds_view(Lg);
  const int lane = threadIdx.x & 63;
  const int rl = lane < R ? lane : 0;          // lanes past R read row 0 and write zeros
  double dv = lane < R ? G[lane + lane * kLdG] : 0.0;
  bool done = lane >= R;
  double dmax0 = 0.0;
  int k = 0;
  for (; k < R; ++k) {
    const int p = pivot_lane(pivot_key(dv, !done, lane));
    const double dp = readlane_d(dv, p);
    if (k == 0) dmax0 = dp;
    if (!(dp > delta * dmax0) || !(dp > 0.0)) break;
    const double piv = sqrt(dp);
    const double rpiv = 1.0 / piv;             // independent of the dot below
    const double sum = G[rl + p * kLdG] - lds_dot<kLdG, kLdG>(Lc + rl, Lc + p, 0, k);
    double c = sum * rpiv;
    if (lane == p) c = piv;
    if (done) c = 0.0;
    Lc[lane + k * kLdG] = c;
    if (lane == p) done = true;
    else if (!done) dv -= c * c;
    wave_lds_sync();
  }
  return k;
}

// Householder QR with column pivoting of K (kA x kB <= 64 x 64, LDS, ld
// kLdG), by waves 0..3 of the work-group (blockDim >= 256; the other waves
// only take part in the barriers).  Lane j owns column j; wave w keeps rows
// 16w..16w+15 of the trailing block in registers, with the rows above the
// current step held at zero, so that the reflector, its dot products and the
// update need no row masks.  Each step writes row s of R and the pivot
// column's Householder vector to K in LDS as they leave the trailing block.
// Columns are not moved: perm[s] is the column taken at step s.  Stops when
// the Frobenius norm of the trailing block is <= tau; the trailing column
// norms are recomputed from the updated entries at every step (no
// downdating, so small trailing norms are not lost to cancellation).  On
// return column perm[s] holds R(0:s, s) in rows 0..s and the Householder
// vector (unit leading entry implicit) below row s; tv[s] is its scalar.
// At most smax steps are taken (a caller that keeps r columns passes r + 1,
// which still tells whether the tolerance needs more).  Two work-group
// barriers per step: one to add up the column norms (and publish row s), one
// to add up the reflector dots.  The step loop is
// unrolled over the sixteen rows of a wave, so row s is a fixed register of
// wave s / 16 and every wave's rows lie wholly above, at or below it.
// scr: 576 doubles of LDS scratch.
__device__ __noinline__ int wg_qrcp(double* Kg, int kA, int kB, double tau, int smax, int* permg, double* tvg,
                                    double* scr) {
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const bool mine = wave < 4;
  const int wv = mine ? wave : 0;
  const int r0 = wv * 16;
  ldsd* K = lds_view(Kg);
  ldsi* perm = lds_view(permg);
  ldsd* tv = lds_view(tvg);
  ldsd* s_nb = lds_view(scr);          // 4 x 64 partial norms
  ldsd* s_db = s_nb + 256;             // 4 x 64 partial dots
  ldsd* s_row = s_nb + 512;            // row s
  ldsd* Kc = K + lane * kLdG;          // this lane's column
  double kt[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) kt[k] = (mine && r0 + k < kA && lane < kB) ? Kc[r0 + k] : 0.0;
  bool done = lane >= kB;
  double pn;
  {
    double p4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 16; ++k) p4[k & 3] = fma(kt[k], kt[k], p4[k & 3]);
    pn = (p4[0] + p4[1]) + (p4[2] + p4[3]);
  }
  const int kmax = min(min(kA, kB), smax);
  int steps = 0;
  bool go = kmax > 0;
  for (int jp = 0; jp < 4 && go; ++jp) {
    const bool w_eq = wv == jp, w_gt = wv > jp;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {      // no early exit, so that the loop unrolls
      const int s = jp * 16 + jj;
      if (s >= kmax) go = false;
      if (!go) continue;
      if (mine) {
        s_nb[wv * 64 + lane] = pn;
        if (w_eq) s_row[lane] = kt[jj];
      }
      __syncthreads();
      const double n2 = ((s_nb[lane] + s_nb[64 + lane]) + s_nb[128 + lane]) + s_nb[192 + lane];
      const double xs = s_row[lane];
      // every lane forms the reflector scalars of its own column while the
      // wave reductions below find the pivot; the pivot lane's are taken
      double bl = 0.0, tl = 0.0, sl = 0.0;
      {
        const double nl = sqrt(n2);
        if (nl > 0.0) {
          bl = xs >= 0 ? -nl : nl;
          const double rb = 1.0 / bl, rd = 1.0 / (xs - bl);      // independent
          tl = (bl - xs) * rb;
          sl = rd;
        }
      }
      const double tot = wave_sum_fixed(done ? 0.0 : n2);
      if (tot <= tau * tau) {                    // same value in every wave
        go = false;
        continue;
      }
      const int p = pivot_lane(pivot_key(n2, !done, lane));
      const double beta = readlane_d(bl, p), tq = readlane_d(tl, p), sc = readlane_d(sl, p);
      // reflector: the pivot column scaled below row s, 1 at row s, 0 above.
      // The pivot lane stores it as the column's Householder vector; the
      // wave's other lanes read it back (broadcast loads).
      if (mine && lane == p) {
        if (w_gt) {
#pragma unroll
          for (int k = 0; k < 16; ++k) Kc[r0 + k] = kt[k] * sc;
        } else if (w_eq) {
#pragma unroll
          for (int k = jj + 1; k < 16; ++k) Kc[r0 + k] = kt[k] * sc;
        }
      }
      wave_lds_sync();
      const ldsd* Kp = K + p * kLdG + r0;
      double v[16];
      if (w_gt) {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = Kp[k];
      } else if (w_eq) {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = k < jj ? 0.0 : (k == jj ? 1.0 : Kp[k]);
      } else {
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = 0.0;
      }
      double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 16; ++k) d4[k & 3] = fma(v[k], kt[k], d4[k & 3]);
      const double pd = (d4[0] + d4[1]) + (d4[2] + d4[3]);
      if (mine) s_db[wv * 64 + lane] = pd;
      if (t == 0) {
        perm[s] = p;
        tv[s] = tq;
      }
      __syncthreads();
      const double dot = ((s_db[lane] + s_db[64 + lane]) + s_db[128 + lane]) + s_db[192 + lane];
      const double wj = tq * dot;
#pragma unroll
      for (int k = 0; k < 16; ++k) kt[k] = fma(-wj, v[k], kt[k]);   // done columns: values unused
      if (w_eq) {                                // row s leaves the trailing block as row s of R
        if (mine && !done) Kc[s] = lane == p ? beta : kt[jj];
        kt[jj] = 0.0;
      }
      if (lane == p) done = true;
      {
        double p4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 16; ++k) p4[k & 3] = fma(kt[k], kt[k], p4[k & 3]);
        pn = (p4[0] + p4[1]) + (p4[2] + p4[3]);
      }
      ++steps;
    }
  }
  // the trailing block of the columns never taken
  if (mine && !done) {
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (r0 + k >= steps && r0 + k < kA) Kc[r0 + k] = kt[k];
  }
  __syncthreads();
  return steps;
}

// Q = H_0 ... H_{r-1} [I_r; 0] (kA x r <= 64 x 32, LDS, ld kLdG) from the
// Householder vectors of Vp (column s holds vector s, unit leading entry
// implicit), by waves 0..3 (blockDim >= 256): lane c forms column c, wave w
// keeps rows 16w..16w+15 in registers; one barrier per reflector to add up
// the four partial dots.  scr: 512 doubles of LDS scratch.
__device__ void wg_form_q(const double* Vg, int kA, int r, const double* tvg, double* Qg, double* scr) {
  const int t = threadIdx.x, wave = t >> 6, c = t & 63;
  const bool mine = wave < 4;
  const int r0 = (mine ? wave : 0) * 16;
  const ldsd* Vp = lds_view(Vg);
  const ldsd* tv = lds_view(tvg);
  ldsd* Q = lds_view(Qg);
  ldsd* s_pd0 = lds_view(scr);         // 2 x 4 x 64 partial dots
  double q[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) q[k] = (r0 + k == c) ? 1.0 : 0.0;
  for (int s = r - 1; s >= 0; --s) {
    double v[16];
    const ldsd* vs = Vp + s * kLdG + r0;
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = vs[k];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = (r0 + k > s && r0 + k < kA) ? v[k] : ((r0 + k == s) ? 1.0 : 0.0);
    double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 16; ++k) d4[k & 3] += v[k] * q[k];
    if (mine) s_pd0[(s & 1) * 256 + wave * 64 + c] = (d4[0] + d4[1]) + (d4[2] + d4[3]);
    __syncthreads();
    const ldsd* pd = s_pd0 + (s & 1) * 256;
    const double w = tv[s] * (((pd[c] + pd[64 + c]) + pd[128 + c]) + pd[192 + c]);
#pragma unroll
    for (int k = 0; k < 16; ++k) q[k] -= w * v[k];
  }
  if (mine && c < r) {
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (r0 + k < kA) Q[r0 + k + c * kLdG] = q[k];
  }
  __syncthreads();
}

struct RecompressOut {
  int rank;
  bool capped;
};

// From the Grams G = A^T A (lds::G) and KC = B^T B (lds::KC), R x R: balance
// the columns (A D, B D^{-1}, D_j = (|b_j| / |a_j|)^{1/2}), factor both Grams by
// pivoted Cholesky (LA, LB), truncate K = LA^T LB by QR with column pivoting
// at tau, and leave the transfer matrices M_U = D LB(:, perm(1:r)) R11^{-1}
// (R x r, ld kMaxCat) in lds::RED and M_V = D^{-1} LA Q1 (R x r, ld kLdG) in
// lds::LB, so that U' = A M_U, V' = B M_V and U' V'^T = A B^T up to the
// discarded trailing block of K.  Waves 0 and 1 factor the two Grams
// concurrently; wave 0 runs the QR; the rest is work-group parallel.
__device__ RecompressOut wg_core_grams(double* Lg, int R, double tau, int rmax) {
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  RecompressOut out{0, false};
  ldsd* L = lds_view(Lg);
  ldsd* G = L + lds::G;
  ldsd* LA = L + lds::LA;
  ldsd* LB = L + lds::LB;
  ldsd* KC = L + lds::KC;
  ldsd* red = L + lds::RED;
  ldsd* vec = L + lds::VEC;     // [0,64) dA [64,128) dB [128,192) D [192,256) 1/D [256,320) tv [320,384) 1/R(j,j)
  int* permg = reinterpret_cast<int*>(Lg + lds::IVEC) + 64;
  const ldsi* perm = lds_view(permg);
  __shared__ int s_k[3];
  for (int j = t; j < R; j += blockDim.x) {
    const double a = G[j + j * kLdG], b = KC[j + j * kLdG];
    // (b / a)^(1/4) from the two fourth roots: no overflow for tiny a
    const bool both = a > 0.0 && b > 0.0;
    const double qa = sqrt(sqrt(a)), qb = sqrt(sqrt(b));
    vec[128 + j] = both ? qb / qa : 1.0;
    vec[192 + j] = both ? qa / qb : 1.0;
    vec[j] = a;
    vec[64 + j] = b;
  }
  wg_sync();
  for (int e = t; e < R * R; e += blockDim.x) {
    const int i = e % R, j = e / R;
    const bool zi = !(vec[i] > 0.0 && vec[64 + i] > 0.0), zj = !(vec[j] > 0.0 && vec[64 + j] > 0.0);
    G[i + j * kLdG] = (zi || zj) ? 0.0 : G[i + j * kLdG] * (vec[128 + i] * vec[128 + j]);
    KC[i + j * kLdG] = (zi || zj) ? 0.0 : KC[i + j * kLdG] * (vec[192 + i] * vec[192 + j]);
  }
  wg_sync();
  const double delta = 1e-15 * R;
  if (wave == 0) {
    const int k = wave_pchol(Lg + lds::G, R, Lg + lds::LA, delta);
    if (lane == 0) s_k[0] = k;
  } else if (wave == 1) {
    const int k = wave_pchol(Lg + lds::KC, R, Lg + lds::LB, delta);
    if (lane == 0) s_k[1] = k;
  }
  wg_sync();
  const int kA = s_k[0], kB = s_k[1];
  if (kA == 0 || kB == 0) return out;
  for (int e = t; e < kA * kB; e += blockDim.x) {
    const int i = e % kA, j = e / kA;
    KC[i + j * kLdG] = lds_dot<1, 1>(LA + i * kLdG, LB + j * kLdG, 0, R);
  }
  wg_sync();
  // rmax + 1 steps tell whether the rank exceeds the cap
  const int rq = wg_qrcp(Lg + lds::KC, kA, kB, tau, rmax + 1, permg, Lg + lds::VEC + 256, Lg + lds::RED);
  const int rr = rq < rmax ? rq : rmax;
  for (int e = t; e < kA * rr; e += blockDim.x) {   // R factor and vectors in pivot order
    const int i = e % kA, c = e / kA;
    G[i + c * kLdG] = KC[i + perm[c] * kLdG];
  }
  wg_sync();
  for (int j = t; j < rr; j += blockDim.x) vec[320 + j] = 1.0 / G[j + j * kLdG];
  wg_form_q(Lg + lds::G, kA, rr, Lg + lds::VEC + 256, Lg + lds::KC, Lg + lds::RED);   // ends with a barrier
  if (t == 0) s_k[2] = rq;
  wg_sync();
  int r = s_k[2];
  if (r > rmax) {
    r = rmax;
    out.capped = true;
  }
  out.rank = r;
  if (r == 0) return out;
  for (int i = t; i < R; i += blockDim.x) {
    for (int j = 0; j < r; ++j) {
      const double x = LB[i + perm[j] * kLdG] - lds_dot<kMaxCat, 1>(red + i, G + j * kLdG, 0, j);
      red[i + j * kMaxCat] = x * vec[320 + j];
    }
    for (int j = 0; j < r; ++j) red[i + j * kMaxCat] *= vec[128 + i];
  }
  wg_sync();
  for (int e = t; e < R * r; e += blockDim.x) {
    const int i = e % R, j = e / R;
    LB[i + j * kLdG] = lds_dot<kLdG, 1>(LA + i, KC + j * kLdG, 0, kA) * vec[192 + i];
  }
  wg_sync();
  return out;
}

// Truncated recompression of A B^T (see the file header).  Outputs
// U (m x r, ldu) and V (n x r, ldv) with r <= rmax.
__device__ __noinline__ RecompressOut wg_recompress(const Cat& A, int64_t m, const Cat& B, int64_t n, double tau,
                                       int rmax, double* U, int64_t ldu, double* V, int64_t ldv,
                                       double* L) {
  const int R = A.cols();
  RecompressOut out{0, false};
  if (R == 0 || m == 0 || n == 0) return out;
  double* red = L + lds::RED;
  wg_atb(A, A, m, L + lds::G, kLdG, red);
  wg_atb(B, B, n, L + lds::KC, kLdG, red);
  out = wg_core_grams(L, R, tau, rmax);
  const int r = out.rank;
  if (r == 0) return out;
  double* LB = L + lds::LB;
  wg_a_times_small(A, m, red, kMaxCat, r, U, ldu, 1.0);
  wg_a_times_small(B, n, LB, kLdG, r, V, ldv, 1.0);
  return out;
}

// -------------------------------------------------------- HODLR products
// Y = sign * F X over the subtree rooted at (d0, j0), F = L^{-1} or U^{-1}
// (or its transpose) held as HODLR: leaves in LUinv/perm, off-diagonal
// blocks in IL / IU.  X and Y point at row 0 of the problem, nc <= 64
// columns.  For every internal node the source child's basis projects X
// (Z = B[src]^T X[src]) and the destination child's basis expands it
// (Y[dst] += B[dst] Z).
enum { kIL = 0, kIU = 1 };

__device__ __noinline__ void wg_hmatvec(const DevPtrs& P, const Item& it, int b, int d0, int64_t j0, int which,
                           bool trans, const double* X, int64_t ldx, int nc, double* Y, int64_t ldy,
                           double sign, double* L) {
  const int t = threadIdx.x;
  const bool src_c1 = (which == kIL) ? !trans : trans;
  const double* Bb = (which == kIL) ? P.IL : P.IU;
  const int32_t* ranks = (which == kIL) ? P.rankL : P.rankU;
  double* Zb = P.Z + it.z0;
  const Node root = P.nodes[node_index(it, d0, j0)];
  double* red = L + lds::RED;
  // projections, level by level
  for (int d = d0; d < it.L; ++d) {
    const int64_t cnt = int64_t(1) << (d - d0);
    const int64_t jb = j0 << (d - d0);
    const double* Bd = Bb + it.lvl0 + int64_t(d) * it.n * kRS;
    if (cnt * kRS * nc >= kWG) {
      // many nodes: one thread per (node, entry), full row loop
      for (int64_t e = t; e < cnt * kRS * nc; e += kWG) {
        const int64_t jj = e / (kRS * nc);
        const int q = int(e % (kRS * nc));
        const int s = q % kRS, c = q / kRS;
        const int64_t nidx = node_index(it, d, jb + jj);
        const int r = ranks[nidx];
        if (s >= r) continue;
        const Node nd = P.nodes[nidx];
        const int64_t n1 = nd.size / 2;
        const int64_t o = src_c1 ? nd.start : nd.start + n1;
        const int64_t ns = src_c1 ? n1 : nd.size - n1;
        double acc = 0;
        for (int64_t i = 0; i < ns; ++i) acc += Bd[o + i + int64_t(s) * it.n] * X[o + i + c * ldx];
        Zb[((cnt - 1) + jj) * kRS * 64 + s + c * kRS] = acc;
      }
    } else {
      for (int64_t jj = 0; jj < cnt; ++jj) {
        const int64_t nidx = node_index(it, d, jb + jj);
        const int r = ranks[nidx];
        const Node nd = P.nodes[nidx];
        const int64_t n1 = nd.size / 2;
        const int64_t o = src_c1 ? nd.start : nd.start + n1;
        const int64_t ns = src_c1 ? n1 : nd.size - n1;
        double* Zn = red + 2048 - kRS * 64;      // staging in the tail of red
        (void)Zn;
        Cat Ab = cat1(Bd + o, it.n, r);
        Cat Xb = cat1(X + o, ldx, nc);
        // write straight into the node's Z slot (global) through LDS
        double* Ct = L + lds::G;                  // r x nc <= 32 x 64
        wg_atb(Ab, Xb, ns, Ct, kLdG, red);
        double* Zs = Zb + ((cnt - 1) + jj) * kRS * 64;
        for (int e = t; e < r * nc; e += kWG) {
          const int s = e % r, c = e / r;
          Zs[s + c * kRS] = Ct[s + c * kLdG];
        }
        wg_sync();
      }
    }
    wg_sync();
  }
  // leaves + expansions, one row per thread
  const int64_t rs = root.start, rn = root.size;
  for (int64_t e = t; e < rn * nc; e += kWG) {
    const int64_t i = rs + e % rn;
    const int c = int(e / rn);
    const int leaf = P.rowleaf[it.row0 + i];
    const Node lf = P.nodes[node_index(it, it.L, leaf)];
    const int li = int(i - lf.start), m = lf.size;
    const int64_t gl = it.leaf0 + leaf;
    const double* Fi = P.LUinv + gl * int64_t(b) * b;
    const int32_t* pm = P.perm + gl * b;
    const int32_t* pmi = P.perminv + gl * b;
    const double* x = X + lf.start + c * ldx;
    double acc = 0;
    if (which == kIL && !trans) {          // L^{-1} P^T x
      acc = x[pm[li]];
      for (int j = 0; j < li; ++j) acc += Fi[li + j * b] * x[pm[j]];
    } else if (which == kIL) {             // P L^{-T} x
      const int q = pmi[li];
      acc = x[q];
      for (int j = q + 1; j < m; ++j) acc += Fi[j + q * b] * x[j];
    } else if (!trans) {                   // U^{-1} x
      for (int j = li; j < m; ++j) acc += Fi[li + j * b] * x[j];
    } else {                               // U^{-T} x
      for (int j = 0; j <= li; ++j) acc += Fi[j + li * b] * x[j];
    }
    for (int d = d0; d < it.L; ++d) {
      const int side = (leaf >> (it.L - d - 1)) & 1;
      const bool dst = src_c1 ? (side == 1) : (side == 0);
      if (!dst) continue;
      const int64_t jn = leaf >> (it.L - d);
      const int64_t nidx = node_index(it, d, jn);
      const int r = ranks[nidx];
      const double* Bd = Bb + it.lvl0 + int64_t(d) * it.n * kRS;
      const int64_t slot = ((int64_t(1) << (d - d0)) - 1) + (jn - (j0 << (d - d0)));
      const double* Zs = Zb + slot * kRS * 64 + c * kRS;
      double s2 = 0;
      for (int s = 0; s < r; ++s) s2 += Bd[i + int64_t(s) * it.n] * Zs[s];
      acc += s2;
    }
    Y[i + c * ldy] = sign * acc;
  }
  wg_sync();
}

// ------------------------------------------------------------ leaf LU
// S = A_leaf - P Q^T, partial-pivoted LU in LDS, inverses of both
// triangular factors.  Returns false on a zero or non-finite pivot.
// Dense leaf of the HODLR LU (Sec. 3.4.1: the diagonal blocks at the finest
// level are factored densely).  S = A_leaf - P Q^T (pending Schur update) is
// factored by Gaussian elimination with partial pivoting, then the inverses of
// its unit lower and upper factors are formed for the solve.  Needs blockDim
// >= 256.
//   elimination: waves 0..3 hold 16 columns each in registers (lane i: row i).
//     At step j the wave owning column j picks the pivot row p (largest
//     |S(i,j)| over rows not yet chosen, compared on its leading 26 bits, ties
//     to the lowest row: within a factor 1 + 2^-14 of the largest, which keeps
//     the growth bound of partial pivoting), forms the multipliers and updates
//     its own later columns; after one work-group barrier the waves to its
//     right update theirs with the pivot row read by readlane.  Rows are not
//     moved: the row chosen at step j is written to position j at the end.
//   inverses: blocked, L^{-1} by one half of the work-group and U^{-1} by the
//     other: 8 x 8 diagonal blocks by substitution, then for block sizes 8, 16,
//     32 the off-diagonal block of each pair, (L^{-1})_21 = -L22^{-1} L21
//     L11^{-1} and (U^{-1})_12 = -U11^{-1} U12 U22^{-1}, by two small products.
__device__ inline bool wg_leaf(const DevPtrs& P, const Item& it, int b, int64_t leaf, const double* PP,
                               const double* PQ, int rp, double* L) {
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  const Node lf = P.nodes[node_index(it, it.L, leaf)];
  const int m = lf.size;
  const int64_t gl = it.leaf0 + leaf;
  double* S = L + lds::S;
  double* LI = L + lds::LI;
  double* UI = L + lds::UI;
  double* PL = L + lds::PL;
  double* QL = L + lds::QL;
  __shared__ int s_perm[kMaxLeaf];
  __shared__ int s_pp[2];
  __shared__ int s_badw[4];
  __shared__ double s_l[2 * 64];
  if (rp > 0) {
    g2l(PP + lf.start, it.n, PL, kMaxLeaf, m, rp);
    g2l(PQ + lf.start, it.n, QL, kMaxLeaf, m, rp);
  }
  g2l(P.Aleaf + gl * int64_t(b) * b, b, S, kLdsLeaf, b, b);
  wg_sync();
  if (rp > 0) {
    // S -= PL QL^T on the FP64 matrix cores: 4 x 4 tiles of 16 x 16, k-steps
    // of 4 over the rp pending columns (zero past rp: those LDS columns are
    // stale); only the m x m block is written
    const ldsd* PL3 = lds_view(PL);
    const ldsd* QL3 = lds_view(QL);
    const int li = lane & 15, lk = lane >> 4;
    for (int tile = wave; tile < 16; tile += int(blockDim.x >> 6)) {
      const int ti = tile & 3, tj = tile >> 2;
      hfde_d4 acc{0.0, 0.0, 0.0, 0.0};
      for (int q0 = 0; q0 < rp; q0 += 4) {
        const int q = q0 + lk;
        const double a = q < rp ? PL3[(ti * 16 + li) + q * kMaxLeaf] : 0.0;
        const double bv = q < rp ? QL3[(tj * 16 + li) + q * kMaxLeaf] : 0.0;
        acc = mfma64(a, bv, acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = ti * 16 + 4 * v + lk, col = tj * 16 + li;
        if (row < m && col < m) S[row + col * kLdsLeaf] -= acc[v];
      }
    }
    wg_sync();
  }
  // ---- elimination
  {
    const bool mine = wave < 4;
    const int c0 = (mine ? wave : 0) * 16;
    double a[16];
#pragma unroll
    for (int k = 0; k < 16; ++k)                // rows and columns past b: identity
      a[k] = (mine && lane < b && c0 + k < b) ? S[lane + (c0 + k) * kLdsLeaf] : (lane == c0 + k ? 1.0 : 0.0);
    bool done = lane >= b;
    int order = lane;
    int bad = 0;
    for (int jp = 0; jp < 4; ++jp) {
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int j = jp * 16 + jj;
        if (j < b) {
          double* lb = s_l + (j & 1) * 64;
          if (wave == jp) {
            const int p = pivot_lane(pivot_key(fabs(a[jj]), !done, lane));
            const double pv = readlane_d(a[jj], p);
            if (!(fabs(pv) > 0.0) || !isfinite(pv)) bad = 1;
            const double ip = 1.0 / pv;
            if (lane == p) {
              done = true;
              order = j;
            }
            const double l = done ? 0.0 : a[jj] * ip;
            if (!done) a[jj] = l;
#pragma unroll
            for (int k = jj + 1; k < 16; ++k) a[k] -= l * readlane_d(a[k], p);
            lb[lane] = l;
            if (lane == 0) {
              s_pp[j & 1] = p;
              s_perm[j] = p;
            }
          }
          __syncthreads();
          if (mine && wave != jp) {              // every wave tracks where each row goes
            const int p = __builtin_amdgcn_readfirstlane(s_pp[j & 1]);
            if (lane == p) {
              done = true;
              order = j;
            }
            if (wave > jp) {
              const double l = lb[lane];
#pragma unroll
              for (int k = 0; k < 16; ++k) a[k] -= l * readlane_d(a[k], p);
            }
          }
        }
      }
    }
    __syncthreads();
    if (mine) {                              // row chosen at step j goes to position j
#pragma unroll
      for (int k = 0; k < 16; ++k) S[order + (c0 + k) * kLdsLeaf] = a[k];
    }
    if (mine && lane == 0) s_badw[wave] = bad;
  }
  for (int e = t; e < 64 * kLdsLeaf; e += blockDim.x) {
    LI[e] = 0.0;
    UI[e] = 0.0;
  }
  wg_sync();
  // ---- inverses (S now holds L\U in pivot order).  Half of the group
  // inverts L, the other half U: the 8 x 8 diagonal blocks by substitution
  // (one column per thread), then the block size doubles and the off-diagonal
  // block of each pair follows from two products (L: X21 = -X22 (L21 X11),
  // U: X12 = -X11 (U12 X22)); pairs of 16 and 32 run on the FP64 matrix cores.
  {
    const int half = blockDim.x >> 1;
    const int grp = t / half, loc = t % half;
    const int gw = loc >> 6, nw = half >> 6;         // wave within the half, waves per half
    const ldsd* S3 = lds_view(S);
    ldsd* X = lds_view(grp == 0 ? LI : UI);
    ldsd* T = lds_view(grp == 0 ? PL : QL);         // products of a level (<= 2048 values)
    if (loc < 64) {                                 // 8 x 8 diagonal blocks, one column per thread
      const int bb = loc >> 3, c = loc & 7, o = bb * 8;
      double x[8];
      if (grp == 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          double v = (k == c) ? 1.0 : 0.0;
#pragma unroll
          for (int q = 0; q < k; ++q) v = fma(-S3[(o + k) + (o + q) * kLdsLeaf], x[q], v);
          x[k] = k < c ? 0.0 : v;
        }
      } else {
        double rd[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) rd[k] = 1.0 / S3[(o + k) + (o + k) * kLdsLeaf];
#pragma unroll
        for (int k = 7; k >= 0; --k) {
          double v = (k == c) ? 1.0 : 0.0;
#pragma unroll
          for (int q = k + 1; q < 8; ++q) v = fma(-S3[(o + k) + (o + q) * kLdsLeaf], x[q], v);
          x[k] = k > c ? 0.0 : v * rd[k];
        }
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) X[(o + k) + (o + c) * kLdsLeaf] = x[k];
    }
    wg_sync();
    // pairs of 8 x 8 blocks: T of pair pi at T + 64 pi, ld 8
    for (int e = loc; e < 256; e += half) {
      const int pi = e >> 6, i = e & 7, c = (e >> 3) & 7, o = pi * 16;
      double v = 0.0;
      if (grp == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q >= c) v = fma(S3[(o + 8 + i) + (o + q) * kLdsLeaf], X[(o + q) + (o + c) * kLdsLeaf], v);
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q <= c) v = fma(S3[(o + i) + (o + 8 + q) * kLdsLeaf], X[(o + 8 + q) + (o + 8 + c) * kLdsLeaf], v);
      }
      T[e] = v;
    }
    wg_sync();
    for (int e = loc; e < 256; e += half) {
      const int pi = e >> 6, i = e & 7, c = (e >> 3) & 7, o = pi * 16;
      const ldsd* Tp = T + pi * 64;
      double v = 0.0;
      if (grp == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q <= i) v = fma(X[(o + 8 + i) + (o + 8 + q) * kLdsLeaf], Tp[q + c * 8], v);
        X[(o + 8 + i) + (o + c) * kLdsLeaf] = -v;
      } else {
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q >= i) v = fma(X[(o + i) + (o + q) * kLdsLeaf], Tp[q + c * 8], v);
        X[(o + i) + (o + 8 + c) * kLdsLeaf] = -v;
      }
    }
    wg_sync();
    // pairs of 16 and 32: 16 x 16 tiles, k-steps of 4; T of pair pi at T + 1024 pi, ld 32
    const int li = lane & 15, lk = lane >> 4;
    for (int sz = 16; sz < 64; sz *= 2) {
      const int nt = sz / 16, tpp = nt * nt, tiles = (64 / (2 * sz)) * tpp, ks = sz / 4;
      for (int tile = gw; tile < tiles; tile += nw) {          // T = L21 X11 or U12 X22
        const int pi = tile / tpp, ti = (tile % tpp) % nt, tj = (tile % tpp) / nt, o = pi * 2 * sz;
        hfde_d4 acc{0.0, 0.0, 0.0, 0.0};
        for (int s4 = 0; s4 < ks; ++s4) {
          const int k = 4 * s4 + lk;
          const double a = grp == 0 ? S3[(o + sz + ti * 16 + li) + (o + k) * kLdsLeaf]
                                    : S3[(o + ti * 16 + li) + (o + sz + k) * kLdsLeaf];
          const double bv = grp == 0 ? X[(o + k) + (o + tj * 16 + li) * kLdsLeaf]
                                     : X[(o + sz + k) + (o + sz + tj * 16 + li) * kLdsLeaf];
          acc = mfma64(a, bv, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) T[pi * 1024 + (ti * 16 + 4 * v + lk) + (tj * 16 + li) * 32] = acc[v];
      }
      wg_sync();
      for (int tile = gw; tile < tiles; tile += nw) {          // X21 = -X22 T or X12 = -X11 T
        const int pi = tile / tpp, ti = (tile % tpp) % nt, tj = (tile % tpp) / nt, o = pi * 2 * sz;
        hfde_d4 acc{0.0, 0.0, 0.0, 0.0};
        for (int s4 = 0; s4 < ks; ++s4) {
          const int k = 4 * s4 + lk;
          const double a = grp == 0 ? X[(o + sz + ti * 16 + li) + (o + sz + k) * kLdsLeaf]
                                    : X[(o + ti * 16 + li) + (o + k) * kLdsLeaf];
          acc = mfma64(a, T[pi * 1024 + k + (tj * 16 + li) * 32], acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = ti * 16 + 4 * v + lk, col = tj * 16 + li;
          if (grp == 0) X[(o + sz + row) + (o + col) * kLdsLeaf] = -acc[v];
          else X[(o + row) + (o + sz + col) * kLdsLeaf] = -acc[v];
        }
      }
      wg_sync();
    }
  }
  double* LUo = P.LU + gl * int64_t(b) * b;
  double* LUi = P.LUinv + gl * int64_t(b) * b;
  for (int e = t; e < b * b; e += blockDim.x) {
    const int i = e % b, j = e / b;
    LUo[e] = S[i + j * kLdsLeaf];
    LUi[e] = (i > j) ? LI[i + j * kLdsLeaf] : UI[i + j * kLdsLeaf];
  }
  if (t < b) {
    P.perm[gl * b + t] = s_perm[t];
    P.perminv[gl * b + s_perm[t]] = t;
  }
  const bool ok = (s_badw[0] | s_badw[1] | s_badw[2] | s_badw[3]) == 0;
  wg_sync();
  return ok;
}

// ------------------------------------ whole factorisation, one work-group per problem
__global__ void __launch_bounds__(kWG) k_factor(DevPtrs P, int b, int rmax) {
  extern __shared__ __align__(16) double Lds[];
  const int item = blockIdx.x;
  const Item it = P.items[item];
  const int t = threadIdx.x;
  int state[kMaxLevels + 1];
  int psrc[kMaxLevels + 1];
  int prank[kMaxLevels + 1];
  int maxrank = 0;
  bool capped = false, bad = false;
  int badleaf = -1;
  const int64_t n = it.n;
  int d = 0;
  int64_t j = 0;
  state[0] = 0;
  psrc[0] = 0;
  prank[0] = 0;
  const double tau = it.tau;
  for (;;) {
    if (t == 0 && (d == it.L || state[d] == 0)) P.rankP[node_index(it, d, j)] = prank[d];
    if (d == it.L) {
      const double* PPs = lvl_ptr(P.PP, it, psrc[d]);
      const double* PQs = lvl_ptr(P.PQ, it, psrc[d]);
      if (!wg_leaf(P, it, b, j, PPs, PQs, prank[d], Lds) && !bad) {
        bad = true;
        badleaf = int(j);
      }
      if (d == 0) break;
      --d;
      j >>= 1;
      continue;
    }
    if (state[d] == 0) {
      state[d] = 1;
      psrc[d + 1] = psrc[d];
      prank[d + 1] = prank[d];
      state[d + 1] = 0;
      ++d;
      j = 2 * j;
      continue;
    }
    const Node nd = P.nodes[node_index(it, d, j)];
    const int64_t o = nd.start, n1 = nd.size / 2, n2 = nd.size - n1;
    const int64_t nidx = node_index(it, d, j);
    double* XL = lvl_ptr(P.XL, it, d);
    double* XR = lvl_ptr(P.XR, it, d);
    double* FL = lvl_ptr(P.FL, it, d);
    double* FU = lvl_ptr(P.FU, it, d);
    double* T1 = lvl_ptr(P.T1, it, d);
    double* T2 = lvl_ptr(P.T2, it, d);
    const double* PPs = lvl_ptr(P.PP, it, psrc[d]);
    const double* PQs = lvl_ptr(P.PQ, it, psrc[d]);
    const int rp = prank[d];
    const int r = it.r;
    if (state[d] == 1) {
      // S12 = U12 V12^T - P1 Q2^T  ->  U12' (T1, c1 rows), V12' (FU, c2 rows)
      Cat A12{XL + o, n, r, 1.0, PPs + o, n, rp, -1.0};
      Cat B12{XR + o + n1, n, r, 1.0, PQs + o + n1, n, rp, 1.0};
      RecompressOut c12 = wg_recompress(A12, n1, B12, n2, tau, rmax, T1 + o, n, FU + o + n1, n, Lds);
      // S21 = U21 V21^T - P2 Q1^T  ->  U21' (FL, c2 rows), V21' (T2, c1 rows)
      Cat A21{XL + o + n1, n, r, 1.0, PPs + o + n1, n, rp, -1.0};
      Cat B21{XR + o, n, r, 1.0, PQs + o, n, rp, 1.0};
      RecompressOut c21 = wg_recompress(A21, n2, B21, n1, tau, rmax, FL + o + n1, n, T2 + o, n, Lds);
      capped |= c12.capped || c21.capped;
      const int r12 = c12.rank, r21 = c21.rank;
      if (t == 0) {
        P.rankU[nidx] = r12;
        P.rankL[nidx] = r21;
      }
      maxrank = max(maxrank, max(r12, r21));
      wg_sync();
      // U~12 = L1^{-1} U12'  (FU, c1 rows);  V~21 = U1^{-T} V21'  (FL, c1 rows)
      if (r12 > 0) wg_hmatvec(P, it, b, d + 1, 2 * j, kIL, false, T1, n, r12, FU, n, 1.0, Lds);
      if (r21 > 0) wg_hmatvec(P, it, b, d + 1, 2 * j, kIU, true, T2, n, r21, FL, n, 1.0, Lds);
      // C = V~21^T U~12 (r21 x r12) in LDS, W = U21' C (T1, c2 rows)
      double* C = Lds + lds::KC;
      int rp2 = 0;
      double* PPn = lvl_ptr(P.PP, it, d + 1);
      double* PQn = lvl_ptr(P.PQ, it, d + 1);
      if (r12 > 0 && r21 > 0) {
        wg_atb(cat1(FL + o, n, r21), cat1(FU + o, n, r12), n1, C, kLdG, Lds + lds::RED);
        wg_a_times_small(cat1(FL + o + n1, n, r21), n2, C, kLdG, r12, T1 + o + n1, n, 1.0);
        if (rp > 0) {
          Cat Ap{PPs + o + n1, n, rp, 1.0, T1 + o + n1, n, r12, 1.0};
          Cat Bp{PQs + o + n1, n, rp, 1.0, FU + o + n1, n, r12, 1.0};
          RecompressOut cp = wg_recompress(Ap, n2, Bp, n2, tau, kRS, PPn + o + n1, n, PQn + o + n1, n, Lds);
          capped |= cp.capped;
          rp2 = cp.rank;
        } else {
          wg_copy_cols(T1 + o + n1, n, n2, r12, PPn + o + n1, n, 1.0);
          wg_copy_cols(FU + o + n1, n, n2, r12, PQn + o + n1, n, 1.0);
          rp2 = r12;
        }
      } else if (rp > 0) {
        wg_copy_cols(PPs + o + n1, n, n2, rp, PPn + o + n1, n, 1.0);
        wg_copy_cols(PQs + o + n1, n, n2, rp, PQn + o + n1, n, 1.0);
        rp2 = rp;
      }
      state[d] = 2;
      psrc[d + 1] = d + 1;
      prank[d + 1] = rp2;
      state[d + 1] = 0;
      ++d;
      j = 2 * j + 1;
      continue;
    }
    // state 2: both children done -> inverse-factor blocks of this node
    const int r12 = P.rankU[nidx], r21 = P.rankL[nidx];
    double* IL = lvl_ptr(P.IL, it, d);
    double* IU = lvl_ptr(P.IU, it, d);
    if (r21 > 0) {
      wg_hmatvec(P, it, b, d + 1, 2 * j + 1, kIL, false, FL, n, r21, IL, n, -1.0, Lds);
      wg_hmatvec(P, it, b, d + 1, 2 * j, kIL, true, FL, n, r21, IL, n, 1.0, Lds);
    }
    if (r12 > 0) {
      wg_hmatvec(P, it, b, d + 1, 2 * j, kIU, false, FU, n, r12, IU, n, -1.0, Lds);
      wg_hmatvec(P, it, b, d + 1, 2 * j + 1, kIU, true, FU, n, r12, IU, n, 1.0, Lds);
    }
    if (d == 0) break;
    --d;
    j >>= 1;
  }
  if (t == 0) {
    int st = P.status[item];
    if (bad) st |= 1;
    if (capped) st |= 4;
    P.status[item] = st;
    P.diag[4 * item + 0] = badleaf;
    P.diag[4 * item + 1] = maxrank;
  }
}

}  // namespace hfde
