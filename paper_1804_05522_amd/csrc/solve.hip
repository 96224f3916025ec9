// Per-step HODLR solve x = U^{-1} L^{-1} b (Sec. 3.5) on gfx950, batched over
// problems, leaves and right-hand sides.
//
// With the HODLR inverses of the triangular factors (see factor.hip), each
// triangular solve is one HODLR matrix product, which is fully parallel:
//   z_node = B[src rows]^T x[src rows]           (projection, per node)
//   y[row] = leaf^{-1} x[leaf] + sum over levels B[row] z_node(row)   (expansion)
// L^{-1}: src = child c1, dst = child c2 (lower blocks);
// U^{-1}: src = c2, dst = c1 (upper blocks).
// Kernels (one work unit = one leaf of one problem, 64 threads = its rows):
//   k_project   per-leaf partial projections for every level,
//   k_reduce    per-node sums of the partials (fixed order: deterministic),
//   k_expand    leaf block + expansions; optionally also the next product's
//               per-leaf projections of the freshly computed rows (fusion of
//               the L^{-1} expansion with the U^{-1} projection).
// Factors may be stored in FP64, FP32 or BF16 (TF); vectors and every
// accumulation stay FP64.
#include "internal.hpp"

namespace hfde {


__device__ inline double ld(const double* p) { return *p; }
__device__ inline double ld(const float* p) { return double(*p); }
__device__ inline double ld(const bf16* p) {
  uint32_t u = uint32_t(p->v) << 16;
  return double(__uint_as_float(u));
}
__device__ inline double cvt(double v) { return v; }
__device__ inline double cvt(float v) { return double(v); }
__device__ inline double cvt(bf16 v) { return double(__uint_as_float(uint32_t(v.v) << 16)); }

// rank of the ancestor at depth `lane` of the work unit's leaf (0 for lanes >= L)
__device__ inline int level_ranks(const int32_t* ranks, const WorkUnit& w, int lane) {
  return lane < w.L ? ranks[w.node0 + ((int64_t(1) << lane) - 1) + (w.leaf >> (w.L - lane))] : 0;
}



// Partial projections of the leaf's rows v (LDS, m x nc, ld 64) onto the
// basis B of every level where the leaf lies in the source child.  The 256
// threads are (level slot, rank index) pairs: slot = t / 32 takes levels
// slot, slot + 8, ...; each thread walks the leaf's rows down one basis
// column (a contiguous 512-byte run), so loads are independent and many are
// in flight.  Partials are level-major: part[(d * leaves + gl) * kRS * nc + s + c kRS].
template <typename TF, int NC>
__device__ void leaf_project(const DevPtrs& P, const Item& it, int leaf, const Node& lf, const TF* Bb,
                             const int32_t* ranks, int src_side, const double* vl, int nc, double* part,
                             int64_t leaves) {
  const int t = threadIdx.x;
  const int slot = t >> 5, s = t & 31;
  const int m = lf.size;
  const int64_t gl = it.leaf0 + leaf;
  // rows in flight: with many columns each entry feeds NC FMAs, so fewer suffice
  constexpr int kRB = NC == 1 ? (sizeof(TF) == 8 ? 32 : 64) : (sizeof(TF) == 8 ? 8 : 16);
  for (int d = slot; d < it.L; d += 8) {
    const int side = (leaf >> (it.L - d - 1)) & 1;
    if (side != src_side) continue;
    const int64_t nidx = node_index(it, d, leaf >> (it.L - d));
    const int r = ranks[nidx];
    const __amdgpu_buffer_rsrc_t R = buf_rsrc(Bb + it.lvl0 + int64_t(d) * it.n * kRS, it.n * kRS * int64_t(sizeof(TF)));
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
#pragma unroll 1
    for (int i0 = 0; i0 < 64; i0 += kRB) {
      TF raw[kRB];
#pragma unroll
      for (int q = 0; q < kRB; ++q) {
        const int i = i0 + q;
        raw[q] = bload(R, (s < r && i < m) ? int((lf.start + i + int64_t(s) * it.n) * sizeof(TF)) : kOob,
                       (const TF*)nullptr);
      }
#pragma unroll
      for (int q = 0; q < kRB; ++q) {
        const double bv = cvt(raw[q]);
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += bv * vl[i0 + q + c * 64];
      }
    }
    if (s >= r) continue;
    double* pout = part + (int64_t(d) * leaves + gl) * int64_t(kRS) * nc + s;
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (c < nc) pout[c * kRS] = acc[c];
  }
}

// Column blocks: blockIdx.y = cb takes columns [cb NC, min(nc, (cb + 1) NC)) of
// a launch's nc; its partials and node sums live in their own regions of the
// work arrays (pstride, zstride apart), laid out as for a launch of its own.
template <typename TF, int NC>
__global__ void __launch_bounds__(256) k_project(DevPtrs P, const WorkUnit* wu, int which, const TF* Bb,
                                                 const double* x, int64_t ldx, int nc, double* part,
                                                 int64_t leaves, int64_t pstride) {
  __shared__ double vl[64 * NC];
  const int cb = blockIdx.y;
  x += int64_t(cb) * NC * ldx;
  part += cb * pstride;
  nc = min(NC, nc - cb * NC);
  const WorkUnit w = wu[blockIdx.x];
  const Item it = P.items[w.item];
  const Node lf = P.nodes[node_index(it, it.L, w.leaf)];
  const int t = threadIdx.x;
  const int32_t* ranks = which == 0 ? P.rankL : P.rankU;
  const int src_side = which == 0 ? 0 : 1;
  for (int e = t; e < 64 * NC; e += blockDim.x) {    // rows past the leaf and columns past nc are zero
    const int i = e % 64, c = e / 64;
    vl[e] = (i < lf.size && c < nc) ? x[it.row0 + lf.start + i + c * ldx] : 0.0;
  }
  __syncthreads();
  leaf_project<TF, NC>(P, it, w.leaf, lf, Bb, ranks, src_side, vl, nc, part, leaves);
}

// z[node] = sum of the per-leaf partials over the leaves of the node's source
// child.  256 threads = groups x (rank, column) entries; each group sums a
// strided subset of the leaves, groups are combined in a fixed order.
__global__ void __launch_bounds__(256) k_reduce(DevPtrs P, const NodeUnit* nu, int which, int nc,
                                                const double* part, double* z, int64_t leaves, int ncb,
                                                int64_t pstride, int64_t zstride) {
  __shared__ double red[256];
  const int cb = blockIdx.y;                 // column block of ncb columns (see k_project)
  part += cb * pstride;
  z += cb * zstride;
  nc = min(ncb, nc - cb * ncb);
  const NodeUnit u = nu[blockIdx.x];
  const Item it = P.items[u.item];
  const int32_t* ranks = which == 0 ? P.rankL : P.rankU;
  const int64_t nidx = node_index(it, u.level, u.j);
  const int r = ranks[nidx];
  const int src_side = which == 0 ? 0 : 1;
  const int64_t span = int64_t(1) << (it.L - u.level - 1);
  const int64_t first = it.leaf0 + (int64_t(u.j) * 2 + src_side) * span;
  const int E = r * nc;
  if (E == 0) return;
  for (int e0 = 0; e0 < E; e0 += 256) {
    const int ecnt = min(256, E - e0);
    const int groups = 256 / ecnt;
    const int t = threadIdx.x;
    const int g = t / ecnt, e = e0 + t % ecnt;
    double acc = 0.0;
    if (g < groups) {
      const int s = e % r, c = e / r;
      const double* pp = part + (int64_t(u.level) * leaves + first) * int64_t(kRS) * nc + s + c * kRS;
      const int64_t stride = int64_t(kRS) * nc;
      // eight independent partial sums: eight loads in flight per thread
      double a8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
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
      const int s = ee % r, c = ee / r;
      z[nidx * int64_t(kRS) * nc + s + c * kRS] = sum;
    }
    __syncthreads();
  }
}

// y = F x on this leaf's rows, F = L^{-1} (which = 0) or U^{-1} (which = 1),
// x read from xin (global), result written to yout; if `next_part` is set,
// also the per-leaf projections of y for U^{-1}.  256 threads = 4 slots x 64
// rows: slot 0 applies the leaf block, slots 1..3 the expansions of levels
// 0, 3, 6, ... / 1, 4, 7, ... / 2, 5, 8, ...; slot sums meet in LDS.
template <typename TF, typename TL, int NC>
__global__ void __launch_bounds__(256) k_expand(DevPtrs P, SolveFactors<TF, TL> F, const WorkUnit* wu, int which,
                                                const double* xin, int64_t ldx, double* yout, int64_t ldy,
                                                int nc, const double* z, double* next_part, int64_t leaves, int b,
                                                int64_t pstride, int64_t zstride) {
  __shared__ double vl[64 * NC];
  __shared__ double yl[4][64 * NC];
  __shared__ double zl[3][kRS * NC];                 // z of a level node, row-major (q, c)
  __shared__ int pm[64];
  const int cb = blockIdx.y;                         // column block (see k_project)
  xin += int64_t(cb) * NC * ldx;
  yout += int64_t(cb) * NC * ldy;
  z += cb * zstride;
  if (next_part != nullptr) next_part += cb * pstride;
  nc = min(NC, nc - cb * NC);
  const WorkUnit w = wu[blockIdx.x];
  const Item it = P.items[w.item];
  const Node lf = P.nodes[node_index(it, it.L, w.leaf)];
  const int t = threadIdx.x;
  const int slot = t >> 6, row = t & 63;
  const int m = lf.size;
  const int64_t gl = it.leaf0 + w.leaf;
  const int32_t* ranks = which == 0 ? P.rankL : P.rankU;
  const TF* Bb = which == 0 ? F.IL : F.IU;
  const int dst_side = which == 0 ? 1 : 0;
  for (int e = t; e < 64 * NC; e += blockDim.x) {    // rows past the leaf and columns past nc are zero
    const int i = e % 64, c = e / 64;
    vl[e] = (i < m && c < nc) ? xin[it.row0 + lf.start + i + c * ldx] : 0.0;
  }
  if (t < 64) pm[t] = t < m ? P.perm[gl * b + t] : 0;
  const int rk = level_ranks(ranks, w, row);
  __syncthreads();
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  if (slot == 0) {
    // leaf block: only the triangle the product uses is fetched, all columns at once
    constexpr int kLB = 8;
    const __amdgpu_buffer_rsrc_t R = buf_rsrc(F.LUinv + gl * int64_t(b) * b, int64_t(b) * b * int64_t(sizeof(TL)));
    if (which == 0 && row < m) {
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = vl[pm[row] + c * 64];     // unit diagonal of L^{-1}
    }
#pragma unroll 1
    for (int j0 = 0; j0 < 64; j0 += kLB) {
      TL raw[kLB];
#pragma unroll
      for (int q = 0; q < kLB; ++q) {
        const int j = j0 + q;
        const bool use = row < m && j < m && (which == 0 ? j < row : j >= row);
        raw[q] = bload(R, use ? int((int64_t(j) * b + row) * sizeof(TL)) : kOob, (const TL*)nullptr);
      }
#pragma unroll
      for (int q = 0; q < kLB; ++q) {
        const double f = cvt(raw[q]);
        const int src = which == 0 ? pm[j0 + q] : j0 + q;
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] += f * vl[src + c * 64];
      }
    }
  } else {
    double* zw = zl[slot - 1];
    int cnt = 0;
    for (int d = 0; d < it.L; ++d) {
      const int side = (w.leaf >> (it.L - d - 1)) & 1;
      if (side != dst_side) continue;
      if ((cnt++ % 3) != slot - 1) continue;
      const int64_t nidx = node_index(it, d, w.leaf >> (it.L - d));
      const int r = __builtin_amdgcn_readlane(rk, d);
      const __amdgpu_buffer_rsrc_t R =
          buf_rsrc(Bb + it.lvl0 + int64_t(d) * it.n * kRS, it.n * kRS * int64_t(sizeof(TF)));
      const double* zn = z + nidx * int64_t(kRS) * nc;
      for (int e = row; e < kRS * NC; e += 64) {
        const int q = e / NC, c = e % NC;
        zw[e] = (q < r && c < nc) ? zn[q + c * kRS] : 0.0;
      }
      wave_lds_sync();
      constexpr int kQB = 8;
#pragma unroll 1
      for (int q0 = 0; q0 < r; q0 += kQB) {
        TF raw[kQB];
#pragma unroll
        for (int q = 0; q < kQB; ++q)
          raw[q] = bload(R, (q0 + q < r && row < m) ? int((lf.start + row + int64_t(q0 + q) * it.n) * sizeof(TF))
                                                     : kOob, (const TF*)nullptr);
#pragma unroll
        for (int q = 0; q < kQB; ++q) {
          const double bv = cvt(raw[q]);
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[c] += bv * zw[(q0 + q) * NC + c];
        }
      }
      wave_lds_sync();
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (c < nc) yl[slot][row + c * 64] = acc[c];
  __syncthreads();
  for (int e = t; e < m * nc; e += blockDim.x) {
    const int i = e % m, c = e / m;
    const double v = (yl[0][i + c * 64] + yl[1][i + c * 64]) + (yl[2][i + c * 64] + yl[3][i + c * 64]);
    vl[i + c * 64] = v;
    yout[it.row0 + lf.start + i + c * ldy] = v;
  }
  __syncthreads();
  if (next_part != nullptr)
    leaf_project<TF, NC>(P, it, w.leaf, lf, F.IU, P.rankU, 1, vl, nc, next_part, leaves);
}

// ------------------------------------------------ single right-hand side
// The time-step solves carry one right-hand side.  There each lane owns one
// row of the leaf, so every basis load is coalesced across the wave.  The
// kernels are built to have few dependent memory round trips per
// work-group: the leaf's geometry comes with its work unit, the ranks of all
// levels arrive in one load (one level per lane), and the basis columns and
// leaf-inverse entries are fetched through buffer loads whose range check
// returns zero without a memory access, so a wave issues every load of a
// level (or of the leaf block) at once and fetches only columns below the
// rank and the triangle of the leaf inverse that the product uses.  Row
// products are summed across the leaf by a transpose through LDS (stride 65:
// conflict-free) in two halves of 16 columns, with four partial sums combined
// in a fixed order.  Levels are dealt round-robin to the waves.
constexpr int kP1Ld = 65;
constexpr int kP1Cols = 16;                    // columns per transpose pass
constexpr int kE1Cols = 16;                    // basis columns loaded per batch in k_expand1
constexpr size_t kSolve1Lds = size_t(4) * kP1Cols * kP1Ld * sizeof(double);
// Partial projections of y (this lane's row value) onto the basis of every
// level where the leaf lies in the source child; rk = level_ranks(...).
template <typename TF>
__device__ void leaf_project1(const WorkUnit& w, const TF* Bb, int rk, int src_side, double yv, double* part,
                              int64_t leaves, double* sm) {
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int m = w.size;
  double* pw = sm + wave * (kP1Cols * kP1Ld);
  int cnt = 0;
  for (int d = 0; d < w.L; ++d) {
    const int side = (w.leaf >> (w.L - d - 1)) & 1;
    if (side != src_side) continue;
    if ((cnt++ & 3) != wave) continue;
    const int r = __builtin_amdgcn_readlane(rk, d);
    const __amdgpu_buffer_rsrc_t R = buf_rsrc(Bb + w.lvl0 + int64_t(d) * w.n * kRS, w.n * kRS * int64_t(sizeof(TF)));
#pragma unroll
    for (int h2 = 0; h2 < kRS / kP1Cols; ++h2) {
      if (kP1Cols * h2 >= r) break;
      TF raw[kP1Cols];
#pragma unroll
      for (int q = 0; q < kP1Cols; ++q) {
        const int qq = kP1Cols * h2 + q;
        raw[q] = bload(R, (qq < r && lane < m) ? int((w.start + lane + int64_t(qq) * w.n) * sizeof(TF)) : kOob,
                       (const TF*)nullptr);
      }
#pragma unroll
      for (int q = 0; q < kP1Cols; ++q) pw[q * kP1Ld + lane] = cvt(raw[q]) * yv;
      wave_lds_sync();
      const int q = lane & (kP1Cols - 1), qq = lane / kP1Cols;     // column, quarter of the rows
      double a4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 16; ++k) a4[k & 3] += pw[q * kP1Ld + qq * 16 + k];
      double v = (a4[0] + a4[1]) + (a4[2] + a4[3]);
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      if (qq == 0 && kP1Cols * h2 + q < r) part[(int64_t(d) * leaves + w.gl) * kRS + kP1Cols * h2 + q] = v;
      wave_lds_sync();
    }
  }
}

template <typename TF>
__global__ void __launch_bounds__(256) k_project1(DevPtrs P, const WorkUnit* wu, int which, const TF* Bb,
                                                  const double* x, double* part, int64_t leaves) {
  extern __shared__ double sm[];
  const WorkUnit w = wu[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int rk = level_ranks(which == 0 ? P.rankL : P.rankU, w, lane);
  const double xv = lane < w.size ? x[w.row0 + w.start + lane] : 0.0;
  leaf_project1<TF>(w, Bb, rk, which == 0 ? 0 : 1, xv, part, leaves, sm);
}

// y = F x on one leaf's rows (F = L^{-1} for which = 0, U^{-1} for which = 1):
// wave 0 applies the leaf block (only the triangle the product uses is
// fetched: strictly lower in pivot order for L^{-1}, upper for U^{-1}), waves
// 1..3 the destination levels round-robin (z_node broadcast from lane s by
// readlane).  If next_part is set, the rows of y are projected for U^{-1} in
// the same launch (dynamic LDS kSolve1Lds; none otherwise).
template <typename TF, typename TL>
__global__ void __launch_bounds__(256) k_expand1(DevPtrs P, SolveFactors<TF, TL> F, const WorkUnit* wu, int which,
                                                 const double* xin, double* yout, const double* z,
                                                 double* next_part, int64_t leaves, int b) {
  extern __shared__ double sm[];
  __shared__ double vl[64];
  __shared__ double xp[64];
  __shared__ double yl[4][64];
  const WorkUnit w = wu[blockIdx.x];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63, row = lane;
  const int m = w.size;
  // ranks of the next projection, loaded early (used after the expansion)
  const int rkU = next_part != nullptr ? level_ranks(P.rankU, w, lane) : 0;
  double acc = 0.0;
  if (wave == 0) {
    constexpr int kLB = sizeof(TL) == 8 ? 32 : 64;    // leaf columns in flight
    const __amdgpu_buffer_rsrc_t R = buf_rsrc(F.LUinv + w.gl * int64_t(b) * b, int64_t(b) * b * int64_t(sizeof(TL)));
    const double xv = row < m ? xin[w.row0 + w.start + row] : 0.0;
    const int pv = row < m ? P.perm[w.gl * b + row] : 0;
    vl[row] = xv;
    wave_lds_sync();
    xp[row] = which == 0 ? vl[pv] : xv;
    wave_lds_sync();
    double a4[4] = {which == 0 && row < m ? xp[row] : 0.0, 0.0, 0.0, 0.0};   // unit diagonal of L^{-1}
#pragma unroll 1
    for (int j0 = 0; j0 < 64; j0 += kLB) {
      TL raw[kLB];
#pragma unroll
      for (int q = 0; q < kLB; ++q) {
        const int j = j0 + q;
        const bool use = row < m && j < m && (which == 0 ? j < row : j >= row);
        raw[q] = bload(R, use ? int((int64_t(j) * b + row) * sizeof(TL)) : kOob, (const TL*)nullptr);
      }
#pragma unroll
      for (int q = 0; q < kLB; ++q) a4[q & 3] += cvt(raw[q]) * xp[j0 + q];
    }
    acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
  } else {
    const int32_t* ranks = which == 0 ? P.rankL : P.rankU;
    const int rk = level_ranks(ranks, w, lane);
    const TF* Bb = which == 0 ? F.IL : F.IU;
    const int dst_side = which == 0 ? 1 : 0;
    double a4[4] = {0.0, 0.0, 0.0, 0.0};
    int cnt = 0;
    for (int d = 0; d < w.L; ++d) {
      const int side = (w.leaf >> (w.L - d - 1)) & 1;
      if (side != dst_side) continue;
      if ((cnt++ % 3) != wave - 1) continue;
      const int64_t nidx = w.node0 + ((int64_t(1) << d) - 1) + (w.leaf >> (w.L - d));
      const int r = __builtin_amdgcn_readlane(rk, d);
      const double zl = lane < kRS ? z[nidx * int64_t(kRS) + lane] : 0.0;
      const double zs = lane < r ? zl : 0.0;
      const __amdgpu_buffer_rsrc_t R =
          buf_rsrc(Bb + w.lvl0 + int64_t(d) * w.n * kRS, w.n * kRS * int64_t(sizeof(TF)));
#pragma unroll
      for (int h2 = 0; h2 < kRS / kE1Cols; ++h2) {      // columns in batches (fewer registers in flight)
        if (kE1Cols * h2 >= r) break;
        TF raw[kE1Cols];
#pragma unroll
        for (int q = 0; q < kE1Cols; ++q) {
          const int qq = kE1Cols * h2 + q;
          raw[q] = bload(R, (qq < r && row < m) ? int((w.start + row + int64_t(qq) * w.n) * sizeof(TF)) : kOob,
                         (const TF*)nullptr);
        }
#pragma unroll
        for (int q = 0; q < kE1Cols; ++q) a4[q & 3] += cvt(raw[q]) * readlane_d(zs, kE1Cols * h2 + q);
      }
    }
    acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
  }
  yl[wave][row] = acc;
  __syncthreads();
  const double y = (yl[0][row] + yl[1][row]) + (yl[2][row] + yl[3][row]);
  if (wave == 0 && row < m) yout[w.row0 + w.start + row] = y;
  if (next_part != nullptr) leaf_project1<TF>(w, F.IU, rkU, 1, row < m ? y : 0.0, next_part, leaves, sm);
}

// ---------------------------------------------------------------- helpers
// out[col * batch + item] = sum of squares of v over the rows of `item`.
__global__ void k_item_norms(DevPtrs P, const double* v, int64_t ld, int nc, double* out) {
  const int item = blockIdx.x, col = blockIdx.y;
  const Item it = P.items[item];
  __shared__ double red[256];
  double acc = 0.0;
  const double* vc = v + it.row0 + int64_t(col) * ld;
  for (int64_t i = threadIdx.x; i < it.n; i += blockDim.x) acc += vc[i] * vc[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[int64_t(col) * gridDim.x + item] = red[0];
}

// z = a x + b y (column blocks), z may alias x or y.
__global__ void k_axpby(int64_t nrows, int nc, double a, const double* x, int64_t ldx, double bco,
                        const double* y, int64_t ldy, double* z, int64_t ldz) {
  const int64_t tot = nrows * nc;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < tot; e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = e % nrows, c = e / nrows;
    const double yv = bco != 0.0 ? bco * y[i + c * ldy] : 0.0;
    z[i + c * ldz] = a * x[i + c * ldx] + yv;
  }
}

// Last refinement update of a time step, with the step's convergence check.
// k_step_update: u += d for every problem (grid: kStepSlices-row slices x
// batch), and per slice the partial sums of d^2 and of the updated u^2, in a
// fixed order.  k_step_check (one work-group): per problem, the slices'
// partials summed in slice order, rel = ||d||_2 / ||u||_2 (a non-finite rel
// counts as +inf), worst[item] = max(worst[item], rel).  The host clears
// worst before a run of steps and compares it with the target afterwards.
constexpr int kStepRows = 2048;   // rows of one k_step_update work-group (256 threads x 8)

__global__ void __launch_bounds__(256) k_step_update(DevPtrs P, double* u, const double* d, double2* part,
                                                     int slices) {
  const Item it = P.items[blockIdx.y];
  const int64_t r0 = int64_t(blockIdx.x) * kStepRows;
  double sd = 0.0, su = 0.0;
  if (r0 < it.n) {
    double* uc = u + it.row0;
    const double* dc = d + it.row0;
    const int64_t r1 = min(it.n, r0 + kStepRows);
#pragma unroll 8
    for (int q = 0; q < kStepRows / 256; ++q) {
      const int64_t i = r0 + q * 256 + threadIdx.x;
      if (i < r1) {
        const double dv = dc[i];
        const double uv = uc[i] + dv;
        uc[i] = uv;
        sd += dv * dv;
        su += uv * uv;
      }
    }
  }
  __shared__ double rd[256], ru[256];
  rd[threadIdx.x] = sd;
  ru[threadIdx.x] = su;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      rd[threadIdx.x] += rd[threadIdx.x + off];
      ru[threadIdx.x] += ru[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) part[int64_t(blockIdx.y) * slices + blockIdx.x] = make_double2(rd[0], ru[0]);
}

// b = E (u + fscale f) per problem (f may be null), E = I + mc (S + S^T)
// scaled by mass: the right-hand side of an implicit Euler step of the
// finite-element scheme (Sec. 2.2.2).  Grid (slices, problems).
__global__ void __launch_bounds__(256) k_step_rhs(DevPtrs P, const double* u, const double* f, double fscale,
                                                  double* b) {
  const Item it = P.items[blockIdx.y];
  const int64_t r0 = int64_t(blockIdx.x) * kStepRows;
  auto v = [&](int64_t i) -> double {
    if (i < 0 || i >= it.n) return 0.0;
    return f ? u[it.row0 + i] + fscale * f[it.row0 + i] : u[it.row0 + i];
  };
  for (int q = 0; q < kStepRows / 256; ++q) {
    const int64_t i = r0 + q * 256 + threadIdx.x;
    if (i >= it.n) break;
    const double vi = v(i);
    b[it.row0 + i] = it.mc != 0.0 ? it.mass * (vi + it.mc * (v(i - 1) + v(i + 1))) : vi;
  }
}

__global__ void __launch_bounds__(256) k_step_check(int batch, const double2* part, int slices, double* worst) {
  for (int item = threadIdx.x; item < batch; item += blockDim.x) {
    double sd = 0.0, su = 0.0;
    for (int q = 0; q < slices; ++q) {
      const double2 v = part[int64_t(item) * slices + q];
      sd += v.x;
      su += v.y;
    }
    double rel = su > 0.0 ? sqrt(sd / su) : (sd > 0.0 ? INFINITY : 0.0);
    if (!(rel == rel)) rel = INFINITY;
    worst[item] = fmax(worst[item], rel);
  }
}

template <typename TF>
__global__ void k_convert(const double* src, TF* dst, int64_t count);

template <>
__global__ void k_convert<float>(const double* src, float* dst, int64_t count) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    dst[i] = float(src[i]);
}

template <>
__global__ void k_convert<bf16>(const double* src, bf16* dst, int64_t count) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x) {
    float f = float(src[i]);
    uint32_t u = __float_as_uint(f);
    uint32_t rounding = 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
    if ((u & 0x7F800000u) == 0x7F800000u) rounding = 0;  // keep inf/nan
    dst[i].v = uint16_t((u + rounding) >> 16);
  }
}

// y = M_H x for the compressed operator itself (leaves dense + off-diagonal
// blocks of every level), one leaf per work unit; used to check the compression.
__global__ void __launch_bounds__(64) k_hmatvec_A_project(DevPtrs P, const WorkUnit* wu, const double* x,
                                                          int64_t ldx, int nc, double* part, int Lmax) {
  // partial projections for both the lower (src c1, basis XR) and upper
  // (src c2, basis XR) blocks: z = XR[src]^T x[src]; slot layout like k_project.
  __shared__ double vl[64 * 64];
  __shared__ double sh[kRS * 65];
  const WorkUnit w = wu[blockIdx.x];
  const Item it = P.items[w.item];
  const Node lf = P.nodes[node_index(it, it.L, w.leaf)];
  const int t = threadIdx.x;
  const int m = lf.size;
  const int64_t gl = it.leaf0 + w.leaf;
  for (int c = 0; c < nc; ++c)
    if (t < m) vl[t + c * 64] = x[it.row0 + lf.start + t + c * ldx];
  __syncthreads();
  for (int d = 0; d < it.L; ++d) {
    const double* Bd = P.XR + it.lvl0 + int64_t(d) * it.n * kRS + lf.start;
    const int r = it.r;
    double* pout = part + (gl * Lmax + d) * int64_t(kRS) * nc;
    for (int c = 0; c < nc; ++c) {
      if (t < m) {
        const double xv = vl[t + c * 64];
        for (int s = 0; s < r; ++s) sh[s * 65 + t] = Bd[t + int64_t(s) * it.n] * xv;
      }
      __syncthreads();
      if (t < r) {
        double acc = 0;
        for (int i = 0; i < m; ++i) acc += sh[t * 65 + i];
        pout[t + c * kRS] = acc;
      }
      __syncthreads();
    }
  }
}

__global__ void k_hmatvec_A_reduce(DevPtrs P, const NodeUnit* nu, int nc, const double* part, double* z,
                                   int Lmax) {
  // z layout: [node][side][s + c*kRS] where side 0 = projection of c1 (feeds A21),
  // side 1 = projection of c2 (feeds A12)
  const NodeUnit u = nu[blockIdx.x];
  const Item it = P.items[u.item];
  const int64_t nidx = node_index(it, u.level, u.j);
  const int r = it.r;
  const int64_t span = int64_t(1) << (it.L - u.level - 1);
  for (int e = threadIdx.x; e < 2 * r * nc; e += blockDim.x) {
    const int side = e / (r * nc);
    const int q = e % (r * nc);
    const int s = q % r, c = q / r;
    const int64_t first = (int64_t(u.j) * 2 + side) * span;
    double acc = 0;
    for (int64_t l = 0; l < span; ++l)
      acc += part[((it.leaf0 + first + l) * Lmax + u.level) * int64_t(kRS) * nc + s + c * kRS];
    z[(nidx * 2 + side) * int64_t(kRS) * nc + s + c * kRS] = acc;
  }
}

__global__ void __launch_bounds__(64) k_hmatvec_A_expand(DevPtrs P, const WorkUnit* wu, const double* x,
                                                         int64_t ldx, double* y, int64_t ldy, int nc,
                                                         const double* z, int b) {
  __shared__ double vl[64 * 64];
  const WorkUnit w = wu[blockIdx.x];
  const Item it = P.items[w.item];
  const Node lf = P.nodes[node_index(it, it.L, w.leaf)];
  const int t = threadIdx.x;
  const int m = lf.size;
  const int64_t gl = it.leaf0 + w.leaf;
  for (int c = 0; c < nc; ++c)
    if (t < m) vl[t + c * 64] = x[it.row0 + lf.start + t + c * ldx];
  __syncthreads();
  if (t >= m) return;
  const double* A = P.Aleaf + gl * int64_t(b) * b;
  for (int c = 0; c < nc; ++c) {
    double acc = 0;
    for (int j = 0; j < m; ++j) acc += A[t + j * b] * vl[j + c * 64];
    for (int d = 0; d < it.L; ++d) {
      const int side = (w.leaf >> (it.L - d - 1)) & 1;
      const int64_t nidx = node_index(it, d, w.leaf >> (it.L - d));
      // row in c2 receives A21 (XL on c2 rows) times the projection of c1 (side 0);
      // row in c1 receives A12 (XL on c1 rows) times the projection of c2 (side 1)
      const double* zn = z + (nidx * 2 + (1 - side)) * int64_t(kRS) * nc + c * kRS;
      const double* Bd = P.XL + it.lvl0 + int64_t(d) * it.n * kRS + lf.start + t;
      for (int s = 0; s < it.r; ++s) acc += Bd[int64_t(s) * it.n] * zn[s];
    }
    y[it.row0 + lf.start + t + c * ldy] = acc;
  }
}

}  // namespace hfde
