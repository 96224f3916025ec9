// HODLR LU factorisation (Sec. 3.5) as a host-scheduled sequence of
// multi-work-group kernels on gfx950.
//
// Same algorithm as factor.hip (block LU with recompressed low-rank Schur
// updates and HODLR inverses of the triangular factors); what changes is the
// execution: the post-order walk runs on the host, and every step of a node
// is one kernel launch over all problems of the batch that share the tree
// (lock-step), spread over as many work-groups as its rows allow:
//   gram    partial A^T B over 1024-row chunks (LDS-staged, 4x4 register tiles)
//   reduce  fixed-order sum of the chunk partials (deterministic)
//   core    one work-group per recompression: balance, pivoted Cholesky of
//           both Grams, core QR with column pivoting, transfer matrices
//   form    row-parallel Y = A * M for the new factors
//   prod    HODLR products with a finished subtree's inverse factors
//           (project / reduce / expand over the subtree's leaves and nodes)
//   leaf    Schur update + pivoted LU + triangular inverses of one leaf.
// For node x (children c1, c2; pending update P Q^T from the ancestors):
//   A : grams of [U12,-P1], [V12,Q2], [U21,-P2], [V21,Q1]; cores S12, S21;
//       forms U12' (T1,c1)  V12' (FU,c2)  U21' (FL,c2)  V21' (T2,c1);
//       products U~12 = L1^{-1} U12' (FU,c1), V~21 = U1^{-T} V21' (FL,c1);
//       C = V~21^T U~12; W = U21' C (T1,c2); gram/core/form of the pending
//       update [P2, W][Q2, V12']^T of c2.
//   B : (after c2) products for the inverse-factor blocks
//       IL(c2) = -L2^{-1} U21', IL(c1) = L1^{-T} V~21,
//       IU(c1) = -U1^{-1} U~12, IU(c2) = U2^{-T} V12'.
#include "internal.hpp"

namespace hfde {

enum ArrId : int8_t { A_XL = 0, A_XR, A_FL, A_FU, A_IL, A_IU, A_T1, A_T2, A_PP, A_PQ };

__device__ inline double* arr_base(const DevPtrs& P, int a) {
  switch (a) {
    case A_XL: return P.XL;
    case A_XR: return P.XR;
    case A_FL: return P.FL;
    case A_FU: return P.FU;
    case A_IL: return P.IL;
    case A_IU: return P.IU;
    case A_T1: return P.T1;
    case A_T2: return P.T2;
    case A_PP: return P.PP;
    default: return P.PQ;
  }
}

// depth whose pending arrays hold the pending update of node (d, j): the
// deepest ancestor-or-self that is a right child (0 if none: no pending).
__host__ __device__ inline int pend_src(int d, int64_t j) {
  if (j == 0) return 0;
  int tz = 0;
  while (((j >> tz) & 1) == 0) ++tz;
  return d - tz;
}

__device__ inline int pend_rank(const DevPtrs& P, const Item& it, int d, int64_t j) {
  const int ps = pend_src(d, j);
  if (ps == 0) return 0;
  return P.rankP[node_index(it, ps, j >> (d - ps))];
}

// One node of one problem.
struct NodeTask {
  int32_t item;
  int32_t d;
  int32_t j;
  int32_t slot;     // index of this task in the step's task list (buffers)
};

// The column-concatenated operands of the phase-A grams and forms.
//   type 0: A12 = [XL_d(c1), -P(c1)]      1: B12 = [XR_d(c2), Q(c2)]
//        2: A21 = [XL_d(c2), -P(c2)]      3: B21 = [XR_d(c1), Q(c1)]
//        4: FL_d(c1) (C = V~21^T U~12, left)   7: FU_d(c1) (right)
//        5: Ap = [P(c2), T1_d(c2)]        6: Bp = [Q(c2), FU_d(c2)]
//        8: FL_d(c2) (W = U21' C)
struct OpRef {
  Cat cat;
  int64_t rows;
};

__device__ inline OpRef op_ref(const DevPtrs& P, const Item& it, int d, int64_t j, int type) {
  const Node nd = P.nodes[node_index(it, d, j)];
  const int64_t o = nd.start, n1 = nd.size / 2, n2 = nd.size - n1, n = it.n;
  const int64_t nidx = node_index(it, d, j);
  const int ps = pend_src(d, j);
  const int rp = pend_rank(P, it, d, j);
  const double* PPs = lvl_ptr(P.PP, it, ps);
  const double* PQs = lvl_ptr(P.PQ, it, ps);
  const double* XL = lvl_ptr(P.XL, it, d);
  const double* XR = lvl_ptr(P.XR, it, d);
  const double* FL = lvl_ptr(P.FL, it, d);
  const double* FU = lvl_ptr(P.FU, it, d);
  const double* T1 = lvl_ptr(P.T1, it, d);
  const int r = it.r, r12 = P.rankU[nidx], r21 = P.rankL[nidx];
  switch (type) {
    case 0: return {Cat{XL + o, n, r, 1.0, PPs + o, n, rp, -1.0}, n1};
    case 1: return {Cat{XR + o + n1, n, r, 1.0, PQs + o + n1, n, rp, 1.0}, n2};
    case 2: return {Cat{XL + o + n1, n, r, 1.0, PPs + o + n1, n, rp, -1.0}, n2};
    case 3: return {Cat{XR + o, n, r, 1.0, PQs + o, n, rp, 1.0}, n1};
    case 4: return {cat1(FL + o, n, r21), n1};
    case 5: return {Cat{PPs + o + n1, n, rp, 1.0, T1 + o + n1, n, r12, 1.0}, n2};
    case 6: return {Cat{PQs + o + n1, n, rp, 1.0, FU + o + n1, n, r12, 1.0}, n2};
    case 7: return {cat1(FU + o, n, r12), n1};
    default: return {cat1(FL + o + n1, n, r21), n2};
  }
}

constexpr int kGramRows = 256;      // default rows per partial (a per-matrix tunable)
constexpr int kFuseRows = 256;      // default largest child of a node whose phase A runs fused (tunable)
constexpr int kGramSub = 64;        // rows staged in LDS at a time
constexpr int kGramLd = 66;         // LDS row stride (16-byte aligned rows, spread banks)
constexpr int kG2 = kMaxCat * kMaxCat;   // one 64 x 64 matrix

// A gram unit: task, pair of operand types (x, y), chunk.
struct GramUnit {
  int32_t task;      // index into the step's task list
  int16_t tx, ty;    // operand types (x^T y)
  int32_t chunk;
  int32_t out;       // output slot (partial index)
};

// ------------------------------------------------ Grams on the matrix cores
constexpr int kStLd = kGramSub + 1;    // column stride (rows) of a staged window in LDS
constexpr int kMaxTW = 5;              // Gram tiles per wave (20 tiles over 4 waves)

// (ti, tj), ti <= tj, of upper-triangle tile s in tj-major order
__device__ inline void sym_tile(int s, int& ti, int& tj) {
  tj = 0;
  while ((tj + 1) * (tj + 2) / 2 <= s) ++tj;
  ti = s - tj * (tj + 1) / 2;
}

// Gram matrices with FP64 matrix-core products.  kTwo: out0 = S0^T S0 and
// out1 = S1^T S1; otherwise out0 = S0^T S1 (symmetric when `same`: S1 is S0).
// Rows [row0, row0 + rows0) of S0 and [row0, row0 + rows1) of S1 enter.  The
// work-group stages windows of kGramSub rows of both operands column-major
// in LDS (st0, st1: kMaxCat x kStLd each), fetching the next window into
// registers while the current one is multiplied; wave w owns the 16 x 16
// output tiles w, w + waves, ... (upper triangle only for a symmetric Gram,
// mirrored on output).  out: ld ldo; zero_rest: zeros over the rest of the
// 64 x 64 block.  Work-groups of 256 or 512 threads.
template <bool kTwo, typename Op>
__device__ void wg_gram_mfma(const Op& S0, const Op& S1, int64_t row0, int64_t rows0, int64_t rows1, bool same,
                             double* out0, double* out1, int ldo, bool zero_rest, double* st0, double* st1) {
  const int nt = blockDim.x, t = threadIdx.x;
  const int l = t & 63, wave = t >> 6, waves = nt >> 6;
  const int c0 = S0.cols(), c1 = S1.cols();
  const int t0 = (c0 + 15) >> 4, t1 = (c1 + 15) >> 4;
  const bool sym0 = kTwo || same;
  const int T0 = sym0 ? t0 * (t0 + 1) / 2 : t0 * t1;
  const int T = kTwo ? T0 + t1 * (t1 + 1) / 2 : T0;
  const bool stage1 = kTwo || !same;
  if (!stage1) rows1 = 0;
  const int64_t most = max(rows0, rows1);
  // this thread stages window row si of columns sc + cstep q
  ldsd* s0 = lds_view(st0);
  ldsd* s1 = lds_view(st1);
  // Unscaled columns are staged (the column pointers are recomputed per
  // window to save registers); the column scales multiply the Gram entries.
  constexpr int kQ = kGramSub * kMaxCat / 256;
  const int si = t % kGramSub, sc = t / kGramSub, cstep = nt / kGramSub;
  auto colptr = [&](const Op& S, int c) {
    double f;
    return S.colp(c, f) + row0;
  };
  auto scale = [&](const Op& S, int c) {
    double f = 0.0;
    (void)S.colp(c, f);
    return f;
  };
  double v0[kQ], v1[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int c = sc + cstep * q;
    v0[q] = (c < c0 && si < rows0) ? colptr(S0, c)[si] : 0.0;
    v1[q] = (stage1 && c < c1 && si < rows1) ? colptr(S1, c)[si] : 0.0;
  }
  hfde_d4 acc[kMaxTW];
#pragma unroll
  for (int q = 0; q < kMaxTW; ++q) acc[q] = hfde_d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t w0 = 0; w0 < most; w0 += kGramSub) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int c = sc + cstep * q;
      if (c < kMaxCat) {
        s0[c * kStLd + si] = v0[q];
        if (stage1) s1[c * kStLd + si] = v1[q];
      }
    }
    __syncthreads();
    if (w0 + kGramSub < most) {
      const int64_t nr = w0 + kGramSub + si;
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const int c = sc + cstep * q;
        v0[q] = (c < c0 && nr < rows0) ? colptr(S0, c)[nr] : 0.0;
        v1[q] = (stage1 && c < c1 && nr < rows1) ? colptr(S1, c)[nr] : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < kMaxTW; ++q) {
      const int tau = wave + q * waves;
      if (tau < T) {
        int ti, tj;
        const bool g1 = kTwo && tau >= T0;
        if (g1) sym_tile(tau - T0, ti, tj);
        else if (sym0) sym_tile(tau, ti, tj);
        else { ti = tau % t0; tj = tau / t0; }
        const ldsd* A = (g1 ? s1 : s0) + (ti * 16 + (l & 15)) * kStLd + (l >> 4);
        const ldsd* B = (kTwo ? (g1 ? s1 : s0) : (same ? s0 : s1)) + (tj * 16 + (l & 15)) * kStLd + (l >> 4);
#pragma unroll
        for (int s4 = 0; s4 < kGramSub; s4 += 4) acc[q] = mfma64(A[s4], B[s4], acc[q]);
      }
    }
  }
  if (zero_rest && !kTwo) {
    const int N0 = same ? c0 : c1;
    for (int e = t; e < kMaxCat * kMaxCat; e += nt) {
      const int i = e % kMaxCat, j = e / kMaxCat;
      if (i >= c0 || j >= N0) out0[i + j * ldo] = 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < kMaxTW; ++q) {
    const int tau = wave + q * waves;
    if (tau < T) {
      int ti, tj;
      const bool g1 = kTwo && tau >= T0;
      if (g1) sym_tile(tau - T0, ti, tj);
      else if (sym0) sym_tile(tau, ti, tj);
      else { ti = tau % t0; tj = tau / t0; }
      double* out = g1 ? out1 : out0;
      const int M = g1 ? c1 : c0, N = (g1 || sym0) ? M : c1;
      const bool mirror = (g1 || sym0) && ti != tj;
      const int j = tj * 16 + (l & 15);
      const double fj0 = scale(S0, j), fj1 = scale(S1, j);
      const double fj = (g1 || !sym0) ? fj1 : fj0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = ti * 16 + 4 * v + (l >> 4);
        if (i < M && j < N) {
          const double fi0 = scale(S0, i), fi1 = scale(S1, i);
          const double g = acc[q][v] * ((g1 ? fi1 : fi0) * fj);
          out[i + j * ldo] = g;
          if (mirror) out[j + i * ldo] = g;
        }
      }
    }
  }
  __syncthreads();
}

// partial[out] = X[chunk rows]^T Y[chunk rows]  (64 x 64, zero padded).
__global__ void __launch_bounds__(256) k_gram_partial(DevPtrs P, const NodeTask* tasks, const GramUnit* units,
                                                      double* partial, int grows) {
  __shared__ __align__(16) double st[2 * kMaxCat * kStLd];
  const GramUnit u = units[blockIdx.x];
  const NodeTask tk = tasks[u.task];
  const Item it = P.items[tk.item];
  const OpRef X = op_ref(P, it, tk.d, tk.j, u.tx);
  const OpRef Y = op_ref(P, it, tk.d, tk.j, u.ty);
  const int64_t r0 = int64_t(u.chunk) * grows;
  const int64_t rows = max<int64_t>(0, min<int64_t>(X.rows, r0 + grows) - r0);
  wg_gram_mfma<false>(X.cat, Y.cat, r0, rows, rows, u.tx == u.ty, partial + int64_t(u.out) * kG2, nullptr, kMaxCat,
                      true, st, st + kMaxCat * kStLd);
}

// G[dst] = sum of partials [first, first + count) in order.
struct ReduceUnit {
  int32_t first;
  int32_t count;
  int32_t dst;
  int32_t pad;
};

__global__ void __launch_bounds__(256) k_gram_reduce(const ReduceUnit* units, const double* partial, double* G) {
  const ReduceUnit u = units[blockIdx.x];
  constexpr int kPer = kG2 / 256;
  double acc[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) acc[k] = 0.0;
  for (int q = 0; q < u.count; ++q) {          // one round trip per partial
    const double* src = partial + int64_t(u.first + q) * kG2 + threadIdx.x;
    double v[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) v[k] = src[k * 256];
#pragma unroll
    for (int k = 0; k < kPer; ++k) acc[k] += v[k];
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) G[int64_t(u.dst) * kG2 + threadIdx.x + k * 256] = acc[k];
}

// Recompression core from two Grams (see wg_recompress): G_A, G_B -> transfer
// matrices M_U (R x r), M_V (R x r) with U' = A M_U, V' = B M_V.
__device__ RecompressOut wg_recompress_core(const double* GAg, const double* GBg, int R, double tau, int rmax,
                                            double* MU, double* MV, double* L) {
  const int t = threadIdx.x;
  RecompressOut out{0, false};
  if (R == 0) return out;
  g2l(GAg, kMaxCat, L + lds::G, kLdG, R, R);
  g2l(GBg, kMaxCat, L + lds::KC, kLdG, R, R);
  wg_sync();
  out = wg_core_grams(L, R, tau, rmax);
  const int r = out.rank;
  const double* red = L + lds::RED;
  const double* LB = L + lds::LB;
  for (int e = t; e < R * r; e += blockDim.x) {
    const int i = e % R, j = e / R;
    MU[i + j * kMaxCat] = red[i + j * kMaxCat];
    MV[i + j * kMaxCat] = LB[i + j * kLdG];
  }
  return out;
}

// Core unit: which recompression of a task (0: S12 -> rankU, 1: S21 -> rankL,
// 2: pending of c2 -> rankP[c2]); grams at G[task*9 + type].
__global__ void __launch_bounds__(kCoreWG) k_core(DevPtrs P, const NodeTask* tasks, const int2* core_units,
                                              const double* G, double* Mbuf, int rmax) {
  extern __shared__ __align__(16) double Lds[];
  const int2 cu = core_units[blockIdx.x];
  const NodeTask tk = tasks[cu.x];
  const int which = cu.y;
  const Item it = P.items[tk.item];
  const int tA = which == 0 ? 0 : (which == 1 ? 2 : 5);
  const OpRef A = op_ref(P, it, tk.d, tk.j, tA);
  const int R = A.cat.cols();
  const double* GA = G + int64_t(tk.slot * 9 + tA) * kG2;
  const double* GB = G + int64_t(tk.slot * 9 + tA + 1) * kG2;
  double* MU = Mbuf + int64_t(tk.slot * 3 + which) * 2 * kMaxCat * kRS;
  double* MV = MU + kMaxCat * kRS;
  const int cap = which == 2 ? kRS : rmax;
  RecompressOut res = wg_recompress_core(GA, GB, R, it.tau, cap, MU, MV, Lds);
  if (threadIdx.x == 0) {
    const int64_t nidx = node_index(it, tk.d, tk.j);
    if (which == 0) P.rankU[nidx] = res.rank;
    else if (which == 1) P.rankL[nidx] = res.rank;
    else P.rankP[node_index(it, tk.d + 1, 2 * int64_t(tk.j) + 1)] = res.rank;
    if (res.capped) atomicOr(&P.status[tk.item], 4);
    atomicMax(&P.diag[4 * tk.item + 1], res.rank);
  }
}

__device__ void wg_form_mfma(const Cat& A, int64_t rows, const double* M, int ldm, int r, double* Y, int64_t ldy,
                             int64_t row0);

// Form unit: rows [chunk*256, +256) of one output of one task.
//   out 0: T1(c1) = A12 M_U12    1: FU(c2) = B12 M_V12    2: FL(c2) = A21 M_U21
//       3: T2(c1) = B21 M_V21    4: T1(c2) = FL(c2) C     5: PP_{d+1}(c2) = Ap M_Up
//       6: PQ_{d+1}(c2) = Bp M_Vp
struct FormUnit {
  int32_t task;
  int32_t out;
  int32_t chunk;
  int32_t pad;
};

__global__ void __launch_bounds__(256) k_form(DevPtrs P, const NodeTask* tasks, const FormUnit* units,
                                              const double* G, const double* Mbuf) {
  __shared__ double Ms[kMaxCat * kRS];
  const FormUnit fu = units[blockIdx.x];
  const NodeTask tk = tasks[fu.task];
  const Item it = P.items[tk.item];
  const int64_t nidx = node_index(it, tk.d, tk.j);
  const Node nd = P.nodes[nidx];
  const int64_t o = nd.start, n1 = nd.size / 2, n = it.n;
  static constexpr int8_t src_type[7] = {0, 1, 2, 3, 8, 5, 6};
  const OpRef A = op_ref(P, it, tk.d, tk.j, src_type[fu.out]);
  const int R = A.cat.cols();
  int r;
  const double* M;
  if (fu.out <= 1) { r = P.rankU[nidx]; M = Mbuf + int64_t(tk.slot * 3 + 0) * 2 * kMaxCat * kRS + (fu.out == 1 ? kMaxCat * kRS : 0); }
  else if (fu.out <= 3) { r = P.rankL[nidx]; M = Mbuf + int64_t(tk.slot * 3 + 1) * 2 * kMaxCat * kRS + (fu.out == 3 ? kMaxCat * kRS : 0); }
  else if (fu.out == 4) { r = P.rankU[nidx]; M = G + int64_t(tk.slot * 9 + 4) * kG2; }
  else { r = P.rankP[node_index(it, tk.d + 1, 2 * int64_t(tk.j) + 1)];
         M = Mbuf + int64_t(tk.slot * 3 + 2) * 2 * kMaxCat * kRS + (fu.out == 6 ? kMaxCat * kRS : 0); }
  // M: R x r with ld kMaxCat (G for C has ld kMaxCat too)
  g2l(M, kMaxCat, Ms, kMaxCat, R, r);
  __syncthreads();
  double* Y;
  int64_t row0;
  switch (fu.out) {
    case 0: Y = lvl_ptr(P.T1, it, tk.d); row0 = o; break;
    case 1: Y = lvl_ptr(P.FU, it, tk.d); row0 = o + n1; break;
    case 2: Y = lvl_ptr(P.FL, it, tk.d); row0 = o + n1; break;
    case 3: Y = lvl_ptr(P.T2, it, tk.d); row0 = o; break;
    case 4: Y = lvl_ptr(P.T1, it, tk.d); row0 = o + n1; break;
    case 5: Y = lvl_ptr(P.PP, it, tk.d + 1); row0 = o + n1; break;
    default: Y = lvl_ptr(P.PQ, it, tk.d + 1); row0 = o + n1; break;
  }
  const int64_t c0 = int64_t(fu.chunk) * 256;
  wg_form_mfma(A.cat, min<int64_t>(256, A.rows - c0), Ms, kMaxCat, r, Y + row0, n, c0);
}

// ------------------------------------------------ fused small-node steps
// For a node whose children hold at most a few hundred rows the Gram chunks,
// their reduction, the core and the forms of a recompression are one
// work-group's job: the group computes both Grams into LDS, runs the core and
// writes the new factors straight from the transfer matrices in LDS.  Phase A
// of such a node is then two launches (plus the subtree products) instead of
// eleven.  Grams and forms run on the FP64 matrix cores in both paths; only
// their summation order differs.

// Y[row0 + i + c ldy] = sum_{k < A.cols()} A(row0 + i, k) M[k + c ldm] for
// i < rows and c < r <= 32, with M in LDS: 16-row tiles of Y (both column
// tiles at once)
// as Y^T = M^T A^T with FP64 matrix-core products.  The M^T operands are the
// same for every tile and stay in registers; the 16 A values of a tile are
// loaded (coalesced over rows) before its products.
__device__ void wg_form_mfma(const Cat& A, int64_t rows, const double* M, int ldm, int r, double* Y, int64_t ldy,
                             int64_t row0) {
  const int R = A.cols();
  const int l = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  const int ks = (R + 3) / 4;
  const bool two = r > 16;
  double ma[kMaxCat / 4], mb[kMaxCat / 4];
#pragma unroll
  for (int s4 = 0; s4 < kMaxCat / 4; ++s4) {
    const int k = 4 * s4 + (l >> 4);
    ma[s4] = k < R ? M[k + (l & 15) * ldm] : 0.0;
    mb[s4] = (two && k < R) ? M[k + (16 + (l & 15)) * ldm] : 0.0;
  }
  for (int64_t rt = wave; rt * 16 < rows; rt += waves) {
    const int64_t i = rt * 16 + (l & 15);
    double av[kMaxCat / 4];
#pragma unroll
    for (int s4 = 0; s4 < kMaxCat / 4; ++s4) {
      const int k = 4 * s4 + (l >> 4);
      av[s4] = (s4 < ks && k < R && i < rows) ? A.at(row0 + i, k) : 0.0;
    }
    hfde_d4 d0{0.0, 0.0, 0.0, 0.0}, d1{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s4 = 0; s4 < kMaxCat / 4; ++s4)
      if (s4 < ks) {
        d0 = mfma64(ma[s4], av[s4], d0);
        if (two) d1 = mfma64(mb[s4], av[s4], d1);
      }
    if (i < rows) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int c = 4 * v + (l >> 4);
        if (c < r) Y[row0 + i + int64_t(c) * ldy] = d0[v];
        if (16 + c < r) Y[row0 + i + int64_t(16 + c) * ldy] = d1[v];
      }
    }
  }
}

// Staging windows of wg_gram_mfma inside the factorisation LDS (region LA,
// which the core only writes after both Grams are in G and KC).
static_assert(2 * kMaxCat * kStLd <= 2 * kMaxCat * kLdG, "gram staging in LA/LB");

__device__ inline void record_rank(const DevPtrs& P, const Item& it, int item, int32_t* slot, RecompressOut res) {
  if (threadIdx.x == 0) {
    *slot = res.rank;
    if (res.capped) atomicOr(&P.status[item], 4);
    atomicMax(&P.diag[4 * item + 1], res.rank);
  }
}

// Phase A, first part, of one node: unit 2k + w recompresses S12 (w = 0:
// U12' -> T1(c1), V12' -> FU(c2)) or S21 (w = 1: U21' -> FL(c2),
// V21' -> T2(c1)) of task k.
__global__ void __launch_bounds__(kCoreWG) k_node_recompress(DevPtrs P, const NodeTask* tasks, int rmax) {
  extern __shared__ __align__(16) double Lf[];
  const NodeTask tk = tasks[blockIdx.x >> 1];
  const int which = blockIdx.x & 1;
  const Item it = P.items[tk.item];
  const int64_t nidx = node_index(it, tk.d, tk.j);
  const Node nd = P.nodes[nidx];
  const int64_t o = nd.start, n1 = nd.size / 2, n = it.n;
  const OpRef A = op_ref(P, it, tk.d, tk.j, 2 * which);
  const OpRef B = op_ref(P, it, tk.d, tk.j, 2 * which + 1);
  const int R = A.cat.cols();
  if (R > 0)
    wg_gram_mfma<true>(A.cat, B.cat, 0, A.rows, B.rows, false, Lf + lds::G, Lf + lds::KC, kLdG, false,
                       Lf + lds::LA, Lf + lds::LA + kMaxCat * kStLd);
  RecompressOut res{0, false};
  if (R > 0) res = wg_core_grams(Lf, R, it.tau, rmax);
  record_rank(P, it, tk.item, which == 0 ? &P.rankU[nidx] : &P.rankL[nidx], res);
  const int r = res.rank;
  if (r == 0) return;
  double* YA = which == 0 ? lvl_ptr(P.T1, it, tk.d) + o : lvl_ptr(P.FL, it, tk.d) + o + n1;
  double* YB = which == 0 ? lvl_ptr(P.FU, it, tk.d) + o + n1 : lvl_ptr(P.T2, it, tk.d) + o;
  wg_form_mfma(A.cat, A.rows, Lf + lds::RED, kMaxCat, r, YA, n, 0);
  wg_form_mfma(B.cat, B.rows, Lf + lds::LB, kLdG, r, YB, n, 0);
}

// Phase A, last part, of one node (after the products U~12, V~21):
// C = V~21^T U~12, W = U21' C -> T1(c2), then the recompression of the
// pending update [P(c2), W][Q(c2), V12']^T of c2 -> PP, PQ at depth d + 1.
__global__ void __launch_bounds__(kCoreWG) k_node_pending(DevPtrs P, const NodeTask* tasks) {
  extern __shared__ __align__(16) double Lf[];
  const NodeTask tk = tasks[blockIdx.x];
  const Item it = P.items[tk.item];
  const int64_t nidx = node_index(it, tk.d, tk.j);
  const Node nd = P.nodes[nidx];
  const int64_t o = nd.start, n1 = nd.size / 2, n = it.n;
  const OpRef F4 = op_ref(P, it, tk.d, tk.j, 4);
  const OpRef F7 = op_ref(P, it, tk.d, tk.j, 7);
  const OpRef F8 = op_ref(P, it, tk.d, tk.j, 8);
  const int r12 = P.rankU[nidx];
  const int c = (F4.cat.cols() > 0 && r12 > 0) ? 1 : 0;
  if (c) {
    wg_gram_mfma<false>(F4.cat, F7.cat, 0, F4.rows, F7.rows, false, Lf + lds::G, nullptr, kLdG, false, Lf + lds::LA,
                        Lf + lds::LA + kMaxCat * kStLd);
    wg_form_mfma(F8.cat, F8.rows, Lf + lds::G, kLdG, r12, lvl_ptr(P.T1, it, tk.d) + o + n1, n, 0);
  }
  else if (r12 > 0) {       // C = 0: W = 0
    double* W = lvl_ptr(P.T1, it, tk.d) + o + n1;
    for (int64_t e = threadIdx.x; e < F8.rows * r12; e += blockDim.x) W[e % F8.rows + (e / F8.rows) * n] = 0.0;
  }
  __syncthreads();          // W is read back below by other threads of the group
  const OpRef Ap = op_ref(P, it, tk.d, tk.j, 5);
  const OpRef Bp = op_ref(P, it, tk.d, tk.j, 6);
  const int R = Ap.cat.cols();
  if (R > 0)
    wg_gram_mfma<true>(Ap.cat, Bp.cat, 0, Ap.rows, Bp.rows, false, Lf + lds::G, Lf + lds::KC, kLdG, false,
                       Lf + lds::LA, Lf + lds::LA + kMaxCat * kStLd);
  RecompressOut res{0, false};
  if (R > 0) res = wg_core_grams(Lf, R, it.tau, kRS);
  record_rank(P, it, tk.item, &P.rankP[node_index(it, tk.d + 1, 2 * int64_t(tk.j) + 1)], res);
  const int r = res.rank;
  if (r == 0) return;
  wg_form_mfma(Ap.cat, Ap.rows, Lf + lds::RED, kMaxCat, r, lvl_ptr(P.PP, it, tk.d + 1) + o + n1, n, 0);
  wg_form_mfma(Bp.cat, Bp.rows, Lf + lds::LB, kLdG, r, lvl_ptr(P.PQ, it, tk.d + 1) + o + n1, n, 0);
}

// --------------------------------------------------- subtree products
// job: Y = sign * F X on the subtree (d0, j0), F in {L^{-1}, L^{-T}, U^{-1}, U^{-T}}
// (which 0/1 = IL/IU, trans), X/Y per-level arrays at level xl/yl of the
// problem, columns = rank of node (rd, rj) in rankU (rk 0) or rankL (rk 1).
struct ProdJob {
  int32_t item;
  int16_t d0;
  int16_t which;
  int32_t j0;
  int16_t trans;
  int8_t xarr, yarr;
  int16_t xlev, ylev;
  int16_t rd;
  int16_t rk;
  int32_t rj;
  int32_t unit0;      // first leaf unit of this job
  int32_t node0;      // first node unit of this job
  double sign;
};

struct ProdUnit {     // leaf unit (leaf = absolute leaf index) or node unit (d, j)
  int32_t job;
  int32_t a;
  int32_t b;
  int32_t pad;
};

__device__ inline int prod_cols(const DevPtrs& P, const Item& it, const ProdJob& jb) {
  const int64_t nidx = node_index(it, jb.rd, jb.rj);
  return jb.rk == 0 ? P.rankU[nidx] : P.rankL[nidx];
}

constexpr int kPNC = kRS;   // columns of a subtree product

constexpr int kSpWaves = 4;          // waves of the subtree-product kernels (256 threads)
constexpr int kSpLd = 65;            // LDS stride of staged 64-row blocks
constexpr size_t kSpProjLds = size_t(64 * kPNC + kSpWaves * kSpLd * kRS) * sizeof(double);
constexpr size_t kSpExpLds = size_t(64 * kPNC + 64 * kSpLd + 64 * kPNC) * sizeof(double);

// Partial projections B_d(leaf rows)^T X(leaf rows) for every subtree level d
// where the leaf is on the source side.  The source levels are dealt
// round-robin to the waves; a wave stages its level's leaf rows of B_d in its
// own LDS slice (one round trip of r loads per lane, zero past the leaf and
// the rank) and forms the r x nc block as 16 x 16 tiles of FP64 matrix-core
// k-steps over the 64 staged rows.
__global__ void __launch_bounds__(256) k_sp_project(DevPtrs P, const ProdJob* jobs, const ProdUnit* units,
                                                    double* part, int Lmax) {
  extern __shared__ double sm[];
  double* xl = sm;
  const ProdUnit u = units[blockIdx.x];
  const ProdJob jb = jobs[u.job];
  const Item it = P.items[jb.item];
  const int leaf = u.a;
  const Node lf = P.nodes[node_index(it, it.L, leaf)];
  const int m = lf.size, nc = prod_cols(P, it, jb);
  const double* X = lvl_ptr(arr_base(P, jb.xarr), it, jb.xlev) + lf.start;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int li = lane & 15, lk = lane >> 4;
  ldsd* Bl = lds_view(sm + 64 * kPNC + wave * kSpLd * kRS);
  const ldsd* xv = lds_view(xl);
  g2l_pad(X, it.n, xl, 64, m, nc, 64, kPNC);
  __syncthreads();
  const bool src_c1 = (jb.which == 0) ? !jb.trans : jb.trans;
  const double* Bb = jb.which == 0 ? P.IL : P.IU;
  const int32_t* ranks = jb.which == 0 ? P.rankL : P.rankU;
  const int nct = nc > 16 ? 2 : 1;
  int cnt = 0;
  for (int d = jb.d0; d < it.L; ++d) {
    const int side = (leaf >> (it.L - d - 1)) & 1;
    if (side != (src_c1 ? 0 : 1)) continue;
    if ((cnt++ % kSpWaves) != wave) continue;
    const int r = ranks[node_index(it, d, leaf >> (it.L - d))];
    const double* Bd = lvl_ptr(const_cast<double*>(Bb), it, d) + lf.start;
    {
      double v[kRS];
#pragma unroll
      for (int q = 0; q < kRS; ++q) v[q] = (q < r && lane < m) ? Bd[lane + int64_t(q) * it.n] : 0.0;
#pragma unroll
      for (int q = 0; q < kRS; ++q) Bl[lane + q * kSpLd] = v[q];
    }
    wave_lds_sync();
    double* po = part + (int64_t(blockIdx.x) * Lmax + d) * kRS * kPNC;
    const int nrt = r > 16 ? 2 : 1;
    for (int rt = 0; rt < nrt; ++rt) {
      hfde_d4 a0{0.0, 0.0, 0.0, 0.0}, a1{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 16; ++s4) {
        const int k = 4 * s4 + lk;
        const double a = Bl[k + (rt * 16 + li) * kSpLd];        // (B_d^T)[row of the block][k]
        a0 = mfma64(a, xv[k + li * 64], a0);
        if (nct > 1) a1 = mfma64(a, xv[k + (16 + li) * 64], a1);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int srow = rt * 16 + 4 * v + lk;
        if (srow < r) {
          if (li < nc) po[srow + li * kRS] = a0[v];
          if (16 + li < nc) po[srow + (16 + li) * kRS] = a1[v];
        }
      }
    }
    wave_lds_sync();
  }
}

// z of one subtree node = sum of its source child's leaf partials (fixed order)
__global__ void __launch_bounds__(256) k_sp_reduce(DevPtrs P, const ProdJob* jobs, const ProdUnit* units,
                                                   const double* part, double* z, int Lmax) {
  __shared__ double red[256];
  const ProdUnit u = units[blockIdx.x];
  const ProdJob jb = jobs[u.job];
  const Item it = P.items[jb.item];
  const int d = u.a, j = u.b;
  const bool src_c1 = (jb.which == 0) ? !jb.trans : jb.trans;
  const int32_t* ranks = jb.which == 0 ? P.rankL : P.rankU;
  const int r = ranks[node_index(it, d, j)];
  const int nc = prod_cols(P, it, jb);
  const int64_t span = int64_t(1) << (it.L - d - 1);
  const int64_t first_leaf = (int64_t(j) * 2 + (src_c1 ? 0 : 1)) * span;
  const int64_t leaf_lo = int64_t(jb.j0) << (it.L - jb.d0);
  const int64_t unit_first = jb.unit0 + (first_leaf - leaf_lo);
  const int64_t slot = ((int64_t(1) << (d - jb.d0)) - 1) + (j - (int64_t(jb.j0) << (d - jb.d0)));
  double* zo = z + (int64_t(jb.node0) + slot) * kRS * kPNC;
  const int E = r * nc;
  const int t = threadIdx.x;
  for (int e0 = 0; e0 < E; e0 += 256) {
    const int ecnt = min(256, E - e0);
    const int groups = 256 / ecnt;
    const int g = t / ecnt, e = e0 + t % ecnt;
    double acc = 0.0;
    if (g < groups) {
      const int s = e % r, c = e / r;
      const double* pp = part + (unit_first * Lmax + d) * kRS * kPNC + s + c * kRS;
      const int64_t stride = int64_t(Lmax) * kRS * kPNC;
      double a8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // eight loads in flight
      int64_t l = g;
      for (; l + 7 * groups < span; l += 8 * groups) {
#pragma unroll
        for (int q = 0; q < 8; ++q) a8[q] += pp[(l + q * groups) * stride];
      }
      for (; l < span; l += groups) a8[0] += pp[l * stride];
      acc = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
    }
    red[t] = acc;
    __syncthreads();
    if (t < ecnt) {
      double sum = 0.0;
      for (int q = 0; q < groups; ++q) sum += red[q * ecnt + t];
      const int ee = e0 + t;
      zo[(ee % r) + (ee / r) * kRS] = sum;
    }
    __syncthreads();
  }
}

// Y rows of the leaf = sign * (leaf op X + sum over destination levels B_d z_d)
// on the FP64 matrix cores.  Wave w owns rows 16w..16w+15 of the leaf and
// both 16-column tiles of the (at most 32) columns.  The leaf op is sixteen
// k-steps of four rows over the staged X rows and inverse factors (the unit
// diagonal of L^{-1} and the triangles taken by masks); each destination
// level adds ceil(r/4) k-steps whose operands, the leaf's rows of B_d and the
// node's z_d, come from range-checked buffer loads, the next level's issued
// before the current level is multiplied.  P L^{-T} x permutes the rows of
// the leaf op's product, which is therefore staged in LDS and gathered before
// the levels are added.
struct SpLevel {
  double a[kRS / 4], z0[kRS / 4], z1[kRS / 4];
  int steps;
};

__global__ void __launch_bounds__(256) k_sp_expand(DevPtrs P, const ProdJob* jobs, const ProdUnit* units,
                                                   const double* z, int b) {
  extern __shared__ double sm[];
  double* xl = sm;                                   // 64 x kPNC, ld 64, zero past the leaf and nc
  double* Fl = xl + 64 * kPNC;                       // 64 x 64, ld kSpLd, zero past the leaf
  double* yl = Fl + 64 * kSpLd;                      // 64 x kPNC, ld 64
  __shared__ int pm[64], pmi[64];
  const ProdUnit u = units[blockIdx.x];
  const ProdJob jb = jobs[u.job];
  const Item it = P.items[jb.item];
  const int leaf = u.a;
  const Node lf = P.nodes[node_index(it, it.L, leaf)];
  const int m = lf.size, nc = prod_cols(P, it, jb);
  const double* X = lvl_ptr(arr_base(P, jb.xarr), it, jb.xlev) + lf.start;
  double* Y = lvl_ptr(arr_base(P, jb.yarr), it, jb.ylev) + lf.start;
  const int t = threadIdx.x, wave = t >> 6, l = t & 63;
  const int li = l & 15, lk = l >> 4;
  const int64_t gl = it.leaf0 + leaf;
  const int i = wave * 16 + li;                      // row of this lane's leaf-op operand
  // destination levels; the first level's operands are fetched while X and
  // the leaf inverse are staged and the leaf op runs
  const bool src_c1 = (jb.which == 0) ? !jb.trans : jb.trans;
  const int dst_side = src_c1 ? 1 : 0;
  const double* Bb = jb.which == 0 ? P.IL : P.IU;
  const int32_t* ranks = jb.which == 0 ? P.rankL : P.rankU;
  auto next_level = [&](int d) {
    for (++d; d < it.L; ++d)
      if (((leaf >> (it.L - d - 1)) & 1) == dst_side) break;
    return d;
  };
  auto fetch = [&](int d, SpLevel& o) {
    const int64_t jn = leaf >> (it.L - d);
    const int r = ranks[node_index(it, d, jn)];
    const int64_t slot = ((int64_t(1) << (d - jb.d0)) - 1) + (jn - (int64_t(jb.j0) << (d - jb.d0)));
    const __amdgpu_buffer_rsrc_t RB =
        buf_rsrc(lvl_ptr(const_cast<double*>(Bb), it, d), it.n * kRS * int64_t(sizeof(double)));
    const __amdgpu_buffer_rsrc_t RZ =
        buf_rsrc(z + (int64_t(jb.node0) + slot) * kRS * kPNC, int64_t(kRS) * kPNC * sizeof(double));
    o.steps = (r + 3) >> 2;
#pragma unroll
    for (int s4 = 0; s4 < kRS / 4; ++s4) {
      const int q = 4 * s4 + lk;
      o.a[s4] = bload(RB, (q < r && i < m) ? int((lf.start + i + int64_t(q) * it.n) * sizeof(double)) : kOob,
                      (const double*)nullptr);
      o.z0[s4] = bload(RZ, (q < r && li < nc) ? int((q + li * kRS) * sizeof(double)) : kOob, (const double*)nullptr);
      o.z1[s4] = bload(RZ, (q < r && 16 + li < nc) ? int((q + (16 + li) * kRS) * sizeof(double)) : kOob,
                       (const double*)nullptr);
    }
  };
  int d = next_level(jb.d0 - 1);
  SpLevel cur, nxt;
  if (d < it.L) fetch(d, cur);
  g2l_pad(X, it.n, xl, 64, m, nc, 64, kPNC);
  g2l_pad(P.LUinv + gl * int64_t(b) * b, b, Fl, kSpLd, m, m, 64, 64);
  if (t < 64) {
    pm[t] = t < m ? P.perm[gl * b + t] : t;
    pmi[t] = t < m ? P.perminv[gl * b + t] : t;
  }
  __syncthreads();
  const bool two = nc > 16;
  // 0: L^{-1} P^T x   1: P L^{-T} x   2: U^{-1} x   3: U^{-T} x
  const int var = 2 * jb.which + jb.trans;
  const double* fa = (var & 1) ? Fl + i * kSpLd : Fl + i;
  const int fs = (var & 1) ? 1 : kSpLd;
  hfde_d4 acc0{0.0, 0.0, 0.0, 0.0}, acc1{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s4 = 0; s4 < 16; ++s4) {
    const int k = 4 * s4 + lk;
    const bool tri = var == 0 ? k < i : (var == 1 ? k > i : (var == 2 ? k >= i : k <= i));
    const double a = tri ? fa[k * fs] : ((var < 2 && k == i) ? 1.0 : 0.0);
    const int xr = var == 0 ? pm[k] : k;
    acc0 = mfma64(a, xl[xr + li * 64], acc0);
    if (two) acc1 = mfma64(a, xl[xr + (16 + li) * 64], acc1);
  }
  if (var == 1) {                                    // rows of L^{-T} x in pivot order: gather
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      yl[wave * 16 + 4 * v + lk + li * 64] = acc0[v];
      yl[wave * 16 + 4 * v + lk + (16 + li) * 64] = acc1[v];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int q = pmi[wave * 16 + 4 * v + lk];
      acc0[v] = yl[q + li * 64];
      acc1[v] = yl[q + (16 + li) * 64];
    }
    __syncthreads();
  }
  while (d < it.L) {
    const int dn = next_level(d);
    if (dn < it.L) fetch(dn, nxt);
#pragma unroll
    for (int s4 = 0; s4 < kRS / 4; ++s4)
      if (s4 < cur.steps) {
        acc0 = mfma64(cur.a[s4], cur.z0[s4], acc0);
        if (two) acc1 = mfma64(cur.a[s4], cur.z1[s4], acc1);
      }
    cur = nxt;
    d = dn;
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    yl[wave * 16 + 4 * v + lk + li * 64] = jb.sign * acc0[v];
    yl[wave * 16 + 4 * v + lk + (16 + li) * 64] = jb.sign * acc1[v];
  }
  __syncthreads();
  for (int e = t; e < m * nc; e += blockDim.x) {
    const int r0 = e % m, c = e / m;
    Y[r0 + int64_t(c) * it.n] = yl[r0 + c * 64];
  }
}

// --------------------------------------------------------------- leaves
// One leaf per unit: the leaf's pending update comes from pend_src.
__global__ void __launch_bounds__(kWG) k_leaf_task(DevPtrs P, const NodeTask* tasks, int b) {
  extern __shared__ __align__(16) double Lds[];
  const NodeTask tk = tasks[blockIdx.x];
  const Item it = P.items[tk.item];
  const int ps = pend_src(tk.d, tk.j);
  const int rp = pend_rank(P, it, tk.d, tk.j);
  if (threadIdx.x == 0) P.rankP[node_index(it, tk.d, tk.j)] = rp;
  const bool ok = wg_leaf(P, it, b, tk.j, lvl_ptr(P.PP, it, ps), lvl_ptr(P.PQ, it, ps), rp, Lds);
  if (!ok && threadIdx.x == 0) {
    if ((atomicOr(&P.status[tk.item], 1) & 1) == 0) P.diag[4 * tk.item] = tk.j;
  }
}

}  // namespace hfde
