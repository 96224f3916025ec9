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

constexpr int kGramRows = 1024;     // rows per partial
constexpr int kGramSub = 32;        // rows staged in LDS at a time
constexpr int kG2 = kMaxCat * kMaxCat;   // one 64 x 64 matrix

// A gram unit: task, pair of operand types (x, y), chunk.
struct GramUnit {
  int32_t task;      // index into the step's task list
  int16_t tx, ty;    // operand types (x^T y)
  int32_t chunk;
  int32_t out;       // output slot (partial index)
};

// partial[out] = X[chunk rows]^T Y[chunk rows]  (64 x 64, zero padded)
__global__ void __launch_bounds__(256) k_gram_partial(DevPtrs P, const NodeTask* tasks, const GramUnit* units,
                                                      double* partial) {
  __shared__ double xs[kGramSub * kMaxCat];
  __shared__ double ys[kGramSub * kMaxCat];
  const GramUnit u = units[blockIdx.x];
  const NodeTask tk = tasks[u.task];
  const Item it = P.items[tk.item];
  const OpRef X = op_ref(P, it, tk.d, tk.j, u.tx);
  const OpRef Y = op_ref(P, it, tk.d, tk.j, u.ty);
  const int M = X.cat.cols(), N = Y.cat.cols();
  const int t = threadIdx.x;
  // thread tile: 4x4 outputs of the 64x64 result
  const int ti = (t % 16) * 4, tj = (t / 16) * 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  const int64_t r0 = int64_t(u.chunk) * kGramRows;
  const int64_t r1 = min<int64_t>(X.rows, r0 + kGramRows);
  for (int64_t s0 = r0; s0 < r1; s0 += kGramSub) {
    const int sr = int(min<int64_t>(kGramSub, r1 - s0));
    __syncthreads();
    for (int e = t; e < kGramSub * kMaxCat; e += 256) {
      const int i = e % kGramSub, c = e / kGramSub;
      xs[e] = (i < sr && c < M) ? X.cat.at(s0 + i, c) : 0.0;
      ys[e] = (i < sr && c < N) ? Y.cat.at(s0 + i, c) : 0.0;
    }
    __syncthreads();
    if (ti < M && tj < N) {
      for (int i = 0; i < sr; ++i) {
        double xv[4], yv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) xv[a] = xs[i + (ti + a) * kGramSub];
#pragma unroll
        for (int b = 0; b < 4; ++b) yv[b] = ys[i + (tj + b) * kGramSub];
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

// G[dst] = sum of partials [first, first + count) in order.
struct ReduceUnit {
  int32_t first;
  int32_t count;
  int32_t dst;
  int32_t pad;
};

__global__ void __launch_bounds__(256) k_gram_reduce(const ReduceUnit* units, const double* partial, double* G) {
  const ReduceUnit u = units[blockIdx.x];
  for (int e = threadIdx.x; e < kG2; e += 256) {
    double s = 0.0;
    for (int q = 0; q < u.count; ++q) s += partial[int64_t(u.first + q) * kG2 + e];
    G[int64_t(u.dst) * kG2 + e] = s;
  }
}

// Recompression core from two Grams (see wg_recompress): G_A, G_B -> transfer
// matrices M_U (R x r), M_V (R x r) with U' = A M_U, V' = B M_V.
__device__ RecompressOut wg_recompress_core(const double* GAg, const double* GBg, int R, double tau, int rmax,
                                            double* MU, double* MV, double* L) {
  const int t = threadIdx.x;
  RecompressOut out{0, false};
  double* G = L + lds::G;
  double* LA = L + lds::LA;
  double* LB = L + lds::LB;
  double* KC = L + lds::KC;
  double* red = L + lds::RED;
  double* vec = L + lds::VEC;
  int* ivec = reinterpret_cast<int*>(L + lds::IVEC);
  if (R == 0) return out;
  for (int e = t; e < R * R; e += blockDim.x) {
    const int i = e % R, j = e / R;
    G[i + j * kLdG] = GAg[i + j * kMaxCat];
    KC[i + j * kLdG] = GBg[i + j * kMaxCat];
  }
  wg_sync();
  for (int j = t; j < R; j += blockDim.x) {
    double a = G[j + j * kLdG], b = KC[j + j * kLdG];
    vec[128 + j] = (a > 0.0 && b > 0.0) ? sqrt(sqrt(b / a)) : 1.0;
    vec[j] = a;
    vec[64 + j] = b;
  }
  wg_sync();
  for (int e = t; e < R * R; e += blockDim.x) {
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
  for (int e = t; e < kA * kB; e += blockDim.x) {
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
  wg_form_q(KC, kA, r, vec + 256, G);
  for (int i = t; i < R; i += blockDim.x) {
    for (int j = 0; j < r; ++j) {
      double x = LB[i + perm[j] * kLdG];
      for (int l = 0; l < j; ++l) x -= red[i + l * kMaxCat] * KC[l + j * kLdG];
      red[i + j * kMaxCat] = x / KC[j + j * kLdG];
    }
    for (int j = 0; j < r; ++j) MU[i + j * kMaxCat] = red[i + j * kMaxCat] * vec[128 + i];
  }
  for (int e = t; e < R * r; e += blockDim.x) {
    const int i = e % R, j = e / R;
    double s = 0;
    for (int q = 0; q < kA; ++q) s += LA[i + q * kLdG] * G[q + j * kLdG];
    MV[i + j * kMaxCat] = s / vec[128 + i];
  }
  wg_sync();
  return out;
}

// Core unit: which recompression of a task (0: S12 -> rankU, 1: S21 -> rankL,
// 2: pending of c2 -> rankP[c2]); grams at G[task*9 + type].
__global__ void __launch_bounds__(kWG) k_core(DevPtrs P, const NodeTask* tasks, const int2* core_units,
                                              const double* G, double* Mbuf, int rmax) {
  extern __shared__ double Lds[];
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
  for (int e = threadIdx.x; e < R * r; e += 256) {
    const int i = e % R, c = e / R;
    Ms[i + c * kMaxCat] = M[i + c * kMaxCat];
  }
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
  const int64_t i = int64_t(fu.chunk) * 256 + threadIdx.x;
  if (i >= A.rows) return;
  double a[kMaxCat];
#pragma unroll
  for (int k = 0; k < kMaxCat; ++k) a[k] = k < R ? A.cat.at(i, k) : 0.0;
  for (int c = 0; c < r; ++c) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxCat; ++k) s += a[k] * Ms[k + c * kMaxCat];
    Y[row0 + i + int64_t(c) * n] = s;
  }
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

// partial projections of the leaf's X rows for every subtree level where the leaf is on the source side
__global__ void __launch_bounds__(256) k_sp_project(DevPtrs P, const ProdJob* jobs, const ProdUnit* units,
                                                    double* part, int Lmax) {
  __shared__ double xl[64 * kPNC];
  const ProdUnit u = units[blockIdx.x];
  const ProdJob jb = jobs[u.job];
  const Item it = P.items[jb.item];
  const int leaf = u.a;
  const Node lf = P.nodes[node_index(it, it.L, leaf)];
  const int m = lf.size, nc = prod_cols(P, it, jb);
  const double* X = lvl_ptr(arr_base(P, jb.xarr), it, jb.xlev) + lf.start;
  const int t = threadIdx.x;
  for (int e = t; e < m * nc; e += 256) {
    const int i = e % m, c = e / m;
    xl[i + c * 64] = X[i + int64_t(c) * it.n];
  }
  __syncthreads();
  const bool src_c1 = (jb.which == 0) ? !jb.trans : jb.trans;
  const double* Bb = jb.which == 0 ? P.IL : P.IU;
  const int32_t* ranks = jb.which == 0 ? P.rankL : P.rankU;
  const int slot = t >> 5, s = t & 31;
  for (int d = jb.d0 + slot; d < it.L; d += 8) {
    const int side = (leaf >> (it.L - d - 1)) & 1;
    if (side != (src_c1 ? 0 : 1)) continue;
    const int r = ranks[node_index(it, d, leaf >> (it.L - d))];
    if (s >= r) continue;
    const double* Bd = lvl_ptr(const_cast<double*>(Bb), it, d) + lf.start + int64_t(s) * it.n;
    double acc[kPNC];
#pragma unroll
    for (int c = 0; c < kPNC; ++c) acc[c] = 0.0;
    for (int i = 0; i < m; ++i) {
      const double bv = Bd[i];
#pragma unroll
      for (int c = 0; c < kPNC; ++c)
        if (c < nc) acc[c] += bv * xl[i + c * 64];
    }
    double* po = part + (int64_t(blockIdx.x) * Lmax + d) * kRS * kPNC + s;
#pragma unroll
    for (int c = 0; c < kPNC; ++c)
      if (c < nc) po[c * kRS] = acc[c];
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
      for (int64_t l = g; l < span; l += groups)
        acc += part[((unit_first + l) * Lmax + d) * kRS * kPNC + s + c * kRS];
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

// Y rows of the leaf = sign * (leaf op X + sum over destination levels B z)
__global__ void __launch_bounds__(128) k_sp_expand(DevPtrs P, const ProdJob* jobs, const ProdUnit* units,
                                                   const double* z, int b) {
  __shared__ double xl[64 * kPNC];
  __shared__ double yl[64 * kPNC];
  __shared__ int pm[64], pmi[64];
  const ProdUnit u = units[blockIdx.x];
  const ProdJob jb = jobs[u.job];
  const Item it = P.items[jb.item];
  const int leaf = u.a;
  const Node lf = P.nodes[node_index(it, it.L, leaf)];
  const int m = lf.size, nc = prod_cols(P, it, jb);
  const double* X = lvl_ptr(arr_base(P, jb.xarr), it, jb.xlev) + lf.start;
  double* Y = lvl_ptr(arr_base(P, jb.yarr), it, jb.ylev) + lf.start;
  const int t = threadIdx.x;
  const int64_t gl = it.leaf0 + leaf;
  const double* Fi = P.LUinv + gl * int64_t(b) * b;
  for (int e = t; e < m * nc; e += 128) {
    const int i = e % m, c = e / m;
    xl[i + c * 64] = X[i + int64_t(c) * it.n];
  }
  if (t < m) {
    pm[t] = P.perm[gl * b + t];
    pmi[t] = P.perminv[gl * b + t];
  }
  __syncthreads();
  const int row = t & 63, half = t >> 6;
  double acc[kPNC];
#pragma unroll
  for (int c = 0; c < kPNC; ++c) acc[c] = 0.0;
  if (row < m) {
    if (half == 0) {
      if (jb.which == 0 && !jb.trans) {            // L^{-1} P^T x
#pragma unroll
        for (int c = 0; c < kPNC; ++c)
          if (c < nc) acc[c] = xl[pm[row] + c * 64];
        for (int jj = 0; jj < row; ++jj) {
          const double f = Fi[row + jj * b];
          const int pj = pm[jj];
#pragma unroll
          for (int c = 0; c < kPNC; ++c)
            if (c < nc) acc[c] += f * xl[pj + c * 64];
        }
      } else if (jb.which == 0) {                   // P L^{-T} x
        const int q = pmi[row];
#pragma unroll
        for (int c = 0; c < kPNC; ++c)
          if (c < nc) acc[c] = xl[q + c * 64];
        for (int jj = q + 1; jj < m; ++jj) {
          const double f = Fi[jj + q * b];
#pragma unroll
          for (int c = 0; c < kPNC; ++c)
            if (c < nc) acc[c] += f * xl[jj + c * 64];
        }
      } else if (!jb.trans) {                       // U^{-1} x
        for (int jj = row; jj < m; ++jj) {
          const double f = Fi[row + jj * b];
#pragma unroll
          for (int c = 0; c < kPNC; ++c)
            if (c < nc) acc[c] += f * xl[jj + c * 64];
        }
      } else {                                      // U^{-T} x
        for (int jj = 0; jj <= row; ++jj) {
          const double f = Fi[jj + row * b];
#pragma unroll
          for (int c = 0; c < kPNC; ++c)
            if (c < nc) acc[c] += f * xl[jj + c * 64];
        }
      }
    } else {
      const bool src_c1 = (jb.which == 0) ? !jb.trans : jb.trans;
      const double* Bb = jb.which == 0 ? P.IL : P.IU;
      const int32_t* ranks = jb.which == 0 ? P.rankL : P.rankU;
      for (int d = jb.d0; d < it.L; ++d) {
        const int side = (leaf >> (it.L - d - 1)) & 1;
        if (side != (src_c1 ? 1 : 0)) continue;
        const int64_t jn = leaf >> (it.L - d);
        const int r = ranks[node_index(it, d, jn)];
        const int64_t slot = ((int64_t(1) << (d - jb.d0)) - 1) + (jn - (int64_t(jb.j0) << (d - jb.d0)));
        const double* zn = z + (int64_t(jb.node0) + slot) * kRS * kPNC;
        const double* Bd = lvl_ptr(const_cast<double*>(Bb), it, d) + lf.start + row;
        for (int s = 0; s < r; ++s) {
          const double bv = Bd[int64_t(s) * it.n];
#pragma unroll
          for (int c = 0; c < kPNC; ++c)
            if (c < nc) acc[c] += bv * zn[s + c * kRS];
        }
      }
    }
  }
  if (half == 1) {
#pragma unroll
    for (int c = 0; c < kPNC; ++c)
      if (c < nc && row < m) yl[row + c * 64] = acc[c];
  }
  __syncthreads();
  if (half == 0 && row < m) {
#pragma unroll
    for (int c = 0; c < kPNC; ++c)
      if (c < nc) Y[row + int64_t(c) * it.n] = jb.sign * (acc[c] + yl[row + c * 64]);
  }
}

// --------------------------------------------------------------- leaves
// One leaf per unit: the leaf's pending update comes from pend_src.
__global__ void __launch_bounds__(kWG) k_leaf_task(DevPtrs P, const NodeTask* tasks, int b) {
  extern __shared__ double Lds[];
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
