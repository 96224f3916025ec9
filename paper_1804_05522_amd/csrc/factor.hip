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
};

__device__ inline Cat cat1(const double* p, int64_t ld, int c) {
  return Cat{p, ld, c, 1.0, p, ld, 0, 0.0};
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

// Pivoted Cholesky of the R x R PSD matrix G (LDS, ld kLdG):  G ~ Lc Lc^T,
// Lc (LDS, R x k, ld kLdG) in original row order.  Right-looking: each step
// takes the largest remaining diagonal entry (wave argmax), forms the column
// and subtracts its outer product from G in parallel.  Stops when the largest
// remaining diagonal entry falls below delta * (largest initial one).
// G is overwritten by the Schur complement.
__device__ int wg_pchol(double* G, int R, double* Lc, double* dv, int* done, double delta) {
  const int t = threadIdx.x;
  __shared__ double s_piv, s_dmax;
  __shared__ int s_p, s_stop;
  for (int i = t; i < R; i += blockDim.x) {
    dv[i] = G[i + i * kLdG];
    done[i] = 0;
  }
  wg_sync();
  if (t < 64) {
    double v = t < R ? dv[t] : -1.0;
    int ix = t;
    wave_argmax(v, ix);
    if (t == 0) s_dmax = v;
  }
  wg_sync();
  const double dmax0 = s_dmax;
  int k = 0;
  for (; k < R; ++k) {
    if (t < 64) {
      double v = (t < R && !done[t]) ? dv[t] : -1.0;
      int ix = t;
      wave_argmax(v, ix);
      if (t == 0) {
        s_stop = (!(v > delta * dmax0) || !(v > 0.0)) ? 1 : 0;
        s_p = ix;
        s_piv = s_stop ? 1.0 : sqrt(v);
        if (!s_stop) done[ix] = 1;
      }
    }
    wg_sync();
    if (s_stop) break;
    const int p = s_p;
    const double piv = s_piv;
    for (int i = t; i < R; i += blockDim.x) {
      double c;
      if (i == p) c = piv;
      else if (done[i]) c = 0.0;
      else c = G[i + p * kLdG] / piv;
      Lc[i + k * kLdG] = c;
    }
    wg_sync();
    for (int e = t; e < R * R; e += blockDim.x) {
      const int i = e % R, j = e / R;
      G[i + j * kLdG] -= Lc[i + k * kLdG] * Lc[j + k * kLdG];
    }
    for (int i = t; i < R; i += blockDim.x) {
      const double c = Lc[i + k * kLdG];
      if (!done[i]) dv[i] -= c * c;
    }
    wg_sync();
  }
  return k;
}

// Householder QR with column pivoting of K (kA x kB, LDS, ld kLdG), stopping
// when the Frobenius norm of the trailing block is <= tau.  On return the
// upper triangle holds R, the Householder vectors sit below the diagonal
// (unit leading entry implicit), tv holds their scalars, perm the column order.
// Column norms are recomputed exactly every step (one wave per column, lanes =
// rows), so tiny trailing norms are not lost to cancellation.
__device__ int wg_qrcp(double* K, int kA, int kB, double tau, int* perm, double* tv, double* cn) {
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  const int nwaves = blockDim.x >> 6;
  __shared__ int s_p, s_stop;
  __shared__ double s_beta, s_tau, s_sc;
  for (int j = t; j < kB; j += blockDim.x) perm[j] = j;
  wg_sync();
  const int kmax = kA < kB ? kA : kB;
  int step = 0;
  for (; step < kmax; ++step) {
    for (int j = step + wave; j < kB; j += nwaves) {
      const double x = (lane >= step && lane < kA) ? K[lane + j * kLdG] : 0.0;
      const double s = wave_sum(x * x);
      if (lane == 0) cn[j] = s;
    }
    wg_sync();
    if (t < 64) {
      double v = (t >= step && t < kB) ? cn[t] : -1.0;
      const double tot = wave_sum((t >= step && t < kB) ? cn[t] : 0.0);
      int ix = t;
      wave_argmax(v, ix);
      if (t == 0) {
        s_stop = (tot <= tau * tau) ? 1 : 0;
        s_p = ix;
      }
    }
    wg_sync();
    if (s_stop) break;
    const int p = s_p;
    if (p != step) {
      for (int i = t; i < kA; i += blockDim.x) {
        const double a = K[i + step * kLdG];
        K[i + step * kLdG] = K[i + p * kLdG];
        K[i + p * kLdG] = a;
      }
      if (t == 0) {
        const int q = perm[step];
        perm[step] = perm[p];
        perm[p] = q;
      }
      wg_sync();
    }
    if (t < 64) {
      const double x0 = K[step + step * kLdG];
      const double xi = (t > step && t < kA) ? K[t + step * kLdG] : 0.0;
      const double s = wave_sum(xi * xi);
      if (t == 0) {
        const double nrm = sqrt(x0 * x0 + s);
        if (nrm == 0.0) {
          s_beta = 0.0; s_tau = 0.0; s_sc = 0.0;
        } else {
          const double beta = x0 >= 0 ? -nrm : nrm;
          s_beta = beta;
          s_tau = (beta - x0) / beta;
          s_sc = 1.0 / (x0 - beta);
        }
      }
    }
    wg_sync();
    for (int i = step + 1 + t; i < kA; i += blockDim.x) K[i + step * kLdG] *= s_sc;
    if (t == 0) {
      K[step + step * kLdG] = s_beta;
      tv[step] = s_tau;
    }
    wg_sync();
    const double tq = s_tau;
    for (int j = step + 1 + wave; j < kB; j += nwaves) {
      const double v = (lane == step) ? 1.0 : ((lane > step && lane < kA) ? K[lane + step * kLdG] : 0.0);
      const double kij = (lane >= step && lane < kA) ? K[lane + j * kLdG] : 0.0;
      const double w = tq * wave_sum(v * kij);
      if (lane >= step && lane < kA) K[lane + j * kLdG] = kij - w * v;
    }
    wg_sync();
  }
  return step;
}

// Q = H_0 ... H_{r-1} [I_r; 0] (kA x r) into Q (LDS, ld kLdG) from the vectors
// left in K by wg_qrcp; one wave per column.
__device__ void wg_form_q(const double* K, int kA, int r, const double* tv, double* Q) {
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63;
  const int nwaves = blockDim.x >> 6;
  for (int e = t; e < kA * r; e += blockDim.x) {
    const int i = e % kA, j = e / kA;
    Q[i + j * kLdG] = (i == j) ? 1.0 : 0.0;
  }
  wg_sync();
  for (int s = r - 1; s >= 0; --s) {
    const double ts = tv[s];
    for (int c = wave; c < r; c += nwaves) {
      const double v = (lane == s) ? 1.0 : ((lane > s && lane < kA) ? K[lane + s * kLdG] : 0.0);
      const double q = (lane >= s && lane < kA) ? Q[lane + c * kLdG] : 0.0;
      const double w = ts * wave_sum(v * q);
      if (lane >= s && lane < kA) Q[lane + c * kLdG] = q - w * v;
    }
    wg_sync();
  }
}

struct RecompressOut {
  int rank;
  bool capped;
};

// Truncated recompression of A B^T (see the file header).  Outputs
// U (m x r, ldu) and V (n x r, ldv) with r <= rmax.
__device__ __noinline__ RecompressOut wg_recompress(const Cat& A, int64_t m, const Cat& B, int64_t n, double tau,
                                       int rmax, double* U, int64_t ldu, double* V, int64_t ldv,
                                       double* L) {
  const int t = threadIdx.x;
  const int R = A.cols();
  RecompressOut out{0, false};
  if (R == 0 || m == 0 || n == 0) return out;
  double* G = L + lds::G;
  double* LA = L + lds::LA;
  double* LB = L + lds::LB;
  double* KC = L + lds::KC;
  double* red = L + lds::RED;
  double* vec = L + lds::VEC;     // [0,64) dA  [64,128) dB  [128,192) D  [192,256) dv  [256,320) tv  [320,384) cn
  int* ivec = reinterpret_cast<int*>(L + lds::IVEC);   // [0,64) done [64,128) perm
  wg_atb(A, A, m, G, kLdG, red);
  wg_atb(B, B, n, KC, kLdG, red);
  for (int j = t; j < R; j += kWG) {
    double a = G[j + j * kLdG], b = KC[j + j * kLdG];
    double Dj = (a > 0.0 && b > 0.0) ? sqrt(sqrt(b / a)) : 1.0;
    vec[128 + j] = Dj;
    vec[j] = a;
    vec[64 + j] = b;
  }
  wg_sync();
  for (int e = t; e < R * R; e += kWG) {
    const int i = e % R, j = e / R;
    const double di = vec[128 + i], dj = vec[128 + j];
    const bool zi = !(vec[i] > 0.0 && vec[64 + i] > 0.0), zj = !(vec[j] > 0.0 && vec[64 + j] > 0.0);
    G[i + j * kLdG] = (zi || zj) ? 0.0 : G[i + j * kLdG] * di * dj;
    KC[i + j * kLdG] = (zi || zj) ? 0.0 : KC[i + j * kLdG] / (di * dj);
  }
  wg_sync();
  const double delta = 1e-15 * R;
  const int kA = wg_pchol(G, R, LA, vec + 192, ivec, delta);
  const int kB = wg_pchol(KC, R, LB, vec + 192, ivec, delta);
  if (kA == 0 || kB == 0) return out;
  // K = LA^T LB (kA x kB)
  for (int e = t; e < kA * kB; e += kWG) {
    const int i = e % kA, j = e / kA;
    double s = 0;
    for (int q = 0; q < R; ++q) s += LA[q + i * kLdG] * LB[q + j * kLdG];
    KC[i + j * kLdG] = s;
  }
  wg_sync();
  int* perm = ivec + 64;
  int r = wg_qrcp(KC, kA, kB, tau, perm, vec + 256, vec + 320);
  if (r > rmax) {
    r = rmax;
    out.capped = true;
  }
  out.rank = r;
  if (r == 0) return out;
  // Q = H_0 ... H_{r-1} [I_r; 0]  (kA x r) into G
  wg_form_q(KC, kA, r, vec + 256, G);
  // M_U = D * LB[:, perm[0:r]] * R11^{-1}  (R x r) into red
  for (int i = t; i < R; i += kWG) {
    for (int j = 0; j < r; ++j) {
      double x = LB[i + perm[j] * kLdG];
      for (int l = 0; l < j; ++l) x -= red[i + l * kMaxCat] * KC[l + j * kLdG];
      red[i + j * kMaxCat] = x / KC[j + j * kLdG];
    }
    for (int j = 0; j < r; ++j) red[i + j * kMaxCat] *= vec[128 + i];
  }
  wg_sync();
  // M_V = D^{-1} * LA * Q  (R x r) into LB
  for (int e = t; e < R * r; e += kWG) {
    const int i = e % R, j = e / R;
    double s = 0;
    for (int q = 0; q < kA; ++q) s += LA[i + q * kLdG] * G[q + j * kLdG];
    LB[i + j * kLdG] = s / vec[128 + i];
  }
  wg_sync();
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
__device__ __noinline__ bool wg_leaf(const DevPtrs& P, const Item& it, int b, int64_t leaf, const double* PP,
                        const double* PQ, int rp, double* L) {
  const int t = threadIdx.x;
  const Node lf = P.nodes[node_index(it, it.L, leaf)];
  const int m = lf.size;
  const int64_t gl = it.leaf0 + leaf;
  double* S = L + lds::S;
  double* LI = L + lds::LI;
  double* UI = L + lds::UI;
  double* PL = L + lds::PL;
  double* QL = L + lds::QL;
  __shared__ int s_p;
  __shared__ int s_bad;
  __shared__ int s_perm[kMaxLeaf];
  for (int e = t; e < m * rp; e += blockDim.x) {
    const int i = e % m, s = e / m;
    PL[i + s * kMaxLeaf] = PP[lf.start + i + int64_t(s) * it.n];
    QL[i + s * kMaxLeaf] = PQ[lf.start + i + int64_t(s) * it.n];
  }
  if (t < b) s_perm[t] = t;
  if (t == 0) s_bad = 0;
  wg_sync();
  const double* A = P.Aleaf + gl * int64_t(b) * b;
  for (int e = t; e < b * b; e += blockDim.x) {
    const int i = e % b, j = e / b;
    double v = A[e];
    if (i < m && j < m)
      for (int s = 0; s < rp; ++s) v -= PL[i + s * kMaxLeaf] * QL[j + s * kMaxLeaf];
    S[i + j * kLdsLeaf] = v;
  }
  wg_sync();
  for (int j = 0; j < b; ++j) {
    if (t < 64) {
      double v = (t >= j && t < b) ? fabs(S[t + j * kLdsLeaf]) : -1.0;
      if (v != v) v = 1e308;   // a NaN pivot candidate is picked and flagged
      int ix = t;
      wave_argmax(v, ix);
      if (t == 0) {
        const double pv = S[ix + j * kLdsLeaf];
        if (!(fabs(pv) > 0.0) || !isfinite(pv)) s_bad = 1;
        s_p = ix;
        if (ix != j) { int q = s_perm[j]; s_perm[j] = s_perm[ix]; s_perm[ix] = q; }
      }
    }
    wg_sync();
    const int p = s_p;
    if (p != j) {
      for (int c = t; c < b; c += blockDim.x) {
        double a = S[j + c * kLdsLeaf];
        S[j + c * kLdsLeaf] = S[p + c * kLdsLeaf];
        S[p + c * kLdsLeaf] = a;
      }
      wg_sync();
    }
    const double piv = S[j + j * kLdsLeaf];
    const double ip = (piv != 0.0) ? 1.0 / piv : 0.0;
    for (int i = j + 1 + t; i < b; i += blockDim.x) S[i + j * kLdsLeaf] *= ip;
    wg_sync();
    const int rem = b - j - 1;
    for (int e = t; e < rem * rem; e += blockDim.x) {
      const int i = j + 1 + e % rem, c = j + 1 + e / rem;
      S[i + c * kLdsLeaf] -= S[i + j * kLdsLeaf] * S[j + c * kLdsLeaf];
    }
    wg_sync();
  }
  // inverses, row by row with 4 threads per dot product: L^{-1} by forward
  // substitution (threads 0..255: column c = t/4), U^{-1} by backward
  // substitution (threads 256..511), one row of each per step.
  {
    const int nt = blockDim.x, half = nt >> 1;
    const int tpd = half >= 64 ? half / 64 : 1;   // threads per dot product: 1, 2 or 4 (blockDim >= 128)
    const int grp = t / half, loc = t % half, c = loc / tpd, q = loc % tpd;
    for (int e = t; e < b * b; e += nt) {
      const int i = e % b, jj = e / b;
      LI[i + jj * kLdsLeaf] = (i == jj) ? 1.0 : 0.0;
      UI[i + jj * kLdsLeaf] = 0.0;
    }
    wg_sync();
    for (int step = 0; step < b; ++step) {
      if (grp == 0) {
        const int i = step;                      // row of L^{-1}
        double s = 0.0;
        if (c < i)
          for (int k = c + q; k < i; k += tpd) s -= S[i + k * kLdsLeaf] * LI[k + c * kLdsLeaf];
        if (tpd > 1) s += __shfl_xor(s, 1);
        if (tpd > 2) s += __shfl_xor(s, 2);
        if (c < i && q == 0) LI[i + c * kLdsLeaf] = s;
      } else {
        const int i = b - 1 - step;              // row of U^{-1}
        double s = 0.0;
        if (c > i && c < b)
          for (int k = i + 1 + q; k <= c; k += tpd) s -= S[i + k * kLdsLeaf] * UI[k + c * kLdsLeaf];
        if (tpd > 1) s += __shfl_xor(s, 1);
        if (tpd > 2) s += __shfl_xor(s, 2);
        if (q == 0 && c >= i && c < b) UI[i + c * kLdsLeaf] = (c == i ? 1.0 : s) / S[i + i * kLdsLeaf];
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
  wg_sync();
  return s_bad == 0;
}

// ------------------------------------------------------------ driver
__global__ void __launch_bounds__(kWG) k_factor(DevPtrs P, int b, int rmax) {
  extern __shared__ double Lds[];
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
