// HODLR construction of M = s I + nu (D+ T + D- T^T) on gfx950.
//
// Sec. 3.4.2: every subdiagonal block of T at every level is a restriction
// of the top-level block, the superdiagonal blocks hold one nonzero, and the
// diagonal scalings act on the outer factors and on the dense leaves.
// Reversing the columns of the top subdiagonal block of T gives (minus) the
// Hankel matrix H[p][q] = g_{p+q+2}, which is positive semidefinite
// (Lemma hadamard-product).  So one symmetric factorisation H ~ W W^T
// serves every off-diagonal block of every level:
//   lower block of node [o, o+n), n1 = floor(n/2):
//     A21[q][p] = -nu d+_{o+n1+q} H[q][n1-1-p]  -  nu d-_{o+n1} [q=0][p=n1-1]
//   upper block:
//     A12[p][q] = -nu d-_{o+p} H[n1-1-p][q]     -  nu d+_{o+n1-1} [p=n1-1][q=0]
// W comes from adaptive cross approximation with diagonal pivoting, which on
// a PSD matrix is a partial pivoted Cholesky; the residual stays PSD, so its
// trace bounds its spectral norm and the stopping test is rigorous.
#include "internal.hpp"

namespace hfde {

// g_0..g_{n+2} by the product recursion g_{k+1} = g_k (k - alpha)/(k + 1)
// (Sec. 3.4.2), evaluated as a blocked multiplicative scan: each thread
// multiplies its segment's factors, one thread scans the segment products,
// then each thread walks its segment again from its prefix.
__global__ void __launch_bounds__(1024) k_gl_weights(DevPtrs P) {
  const Item it = P.items[blockIdx.x];
  const int64_t cnt = it.n + 3;           // g_0 .. g_{n+2}
  double* g = P.g + it.g0;
  __shared__ double seg[1024];
  const int nt = blockDim.x;
  const int64_t per = (cnt + nt - 1) / nt;
  const int64_t k0 = int64_t(threadIdx.x) * per;
  const int64_t k1 = k0 + per < cnt ? k0 + per : cnt;
  double prod = 1.0;
  for (int64_t k = k0; k < k1; ++k) prod *= (double(k) - it.alpha) / double(k + 1);
  seg[threadIdx.x] = prod;
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = 1.0;
    for (int t = 0; t < nt; ++t) {
      double v = seg[t];
      seg[t] = run;
      run *= v;
    }
  }
  __syncthreads();
  double gk = seg[threadIdx.x];            // = g_{k0}
  for (int64_t k = k0; k < k1; ++k) {
    g[k] = gk;
    gk *= (double(k) - it.alpha) / double(k + 1);
  }
}

template <typename T>
__device__ inline void block_reduce_max_sum(T& vmax, int& imax, T& vsum, T* s_v, int* s_i, T* s_s) {
  // one value per thread in, block-wide max (with index) and sum out (all threads)
  const int t = threadIdx.x;
  s_v[t] = vmax;
  s_i[t] = imax;
  s_s[t] = vsum;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if (t < off) {
      if (s_v[t + off] > s_v[t] || (s_v[t + off] == s_v[t] && s_i[t + off] < s_i[t])) {
        s_v[t] = s_v[t + off];
        s_i[t] = s_i[t + off];
      }
      s_s[t] += s_s[t + off];
    }
    __syncthreads();
  }
  vmax = s_v[0];
  imax = s_i[0];
  vsum = s_s[0];
  __syncthreads();
}

// Adaptive cross approximation with diagonal pivoting of H[p][q] = g_{p+q+2},
// p, q < nh.  Column t: pivot p* = argmax of the residual diagonal,
// W[:,t] = (H[:,p*] - W[:, :t] W[p*, :t]^T) / sqrt(d[p*]).  Stops when the
// residual trace <= tolH, or at kRS - 1 columns (flagged).  Also derives the
// truncation tolerances from eps: ||M||_2 >= max_i M_ii = s + nu alpha max(d+ + d-).
__global__ void __launch_bounds__(512) k_hankel_aca(DevPtrs P, double eps) {
  Item& itr = P.items[blockIdx.x];
  const Item it = itr;
  const int nt = blockDim.x;
  const int t0 = threadIdx.x;
  __shared__ double s_v[512];
  __shared__ int s_i[512];
  __shared__ double s_s[512];
  __shared__ double wp[kRS];
  __shared__ int pivots[kRS];
  const double* g = P.g + it.g0;
  const double* dp = P.dplus + it.row0;
  const double* dm = P.dminus + it.row0;
  // tolerances
  double lmax = 0.0, lsum = 0.0;
  int li = 0;
  double mp = 0.0, mm = 0.0;
  for (int64_t i = t0; i < it.n; i += nt) {
    double s = dp[i] + dm[i];
    if (s > lmax) { lmax = s; li = int(i); }
    mp = fmax(mp, dp[i]);
    mm = fmax(mm, dm[i]);
  }
  block_reduce_max_sum(lmax, li, lsum, s_v, s_i, s_s);
  double dsum_max = lmax;
  double dpm = fmax(mp, mm);
  li = 0; lsum = 0.0;
  block_reduce_max_sum(dpm, li, lsum, s_v, s_i, s_s);
  const double mlow = it.shift + it.nu * it.alpha * dsum_max;
  const double tau = eps * mlow;
  const double scale = it.nu * dpm;
  const double tolH = scale > 0.0 ? tau / scale : 1e300;
  const int64_t nh = it.nh;
  double* W = P.W + it.w0;
  double* d = P.T1 + it.lvl0;             // residual diagonal (scratch)
  for (int64_t p = t0; p < nh; p += nt) d[p] = g[2 * p + 2];
  __syncthreads();
  int k = 0;
  bool capped = false;
  for (;;) {
    double vmax = -1.0, vsum = 0.0;
    int imax = 0;
    for (int64_t p = t0; p < nh; p += nt) {
      double v = d[p];
      vsum += v > 0.0 ? v : 0.0;
      if (v > vmax) { vmax = v; imax = int(p); }
    }
    block_reduce_max_sum(vmax, imax, vsum, s_v, s_i, s_s);
    if (vsum <= 0.5 * tolH || vmax <= 0.0) break;
    if (k >= kRS - 1) { capped = true; break; }
    const int pv = imax;
    if (t0 < k) wp[t0] = W[pv + int64_t(t0) * nh];
    if (t0 == 0) pivots[k] = pv;
    __syncthreads();
    const double piv = sqrt(vmax);
    for (int64_t q = t0; q < nh; q += nt) {
      double c = g[q + pv + 2];
      for (int s = 0; s < k; ++s) c -= W[q + int64_t(s) * nh] * wp[s];
      bool done = false;
      for (int s = 0; s <= k; ++s) done |= (pivots[s] == int(q));
      double w = done ? 0.0 : c / piv;
      if (q == pv) w = piv;
      W[q + int64_t(k) * nh] = w;
      d[q] = done || q == pv ? 0.0 : d[q] - w * w;
    }
    __syncthreads();
    ++k;
  }
  if (t0 == 0) {
    itr.k = k;
    itr.r = (scale > 0.0) ? k + 1 : 0;
    itr.tau = tau;
    itr.tolH = tolH;
    P.diag[4 * blockIdx.x + 3] = k;
    if (capped) P.status[blockIdx.x] |= 4;
  }
}

// Truncation of the Hankel factor to the 2-norm eps-rank.  The trace-stopped
// cross approximation leaves ||H - W W^T||_2 <= trace <= tolH/2 but keeps
// columns whose directions carry less than that: the eigenvalues of W W^T are
// those of G = W^T W (k x k).  G is formed in LDS (128-row chunks, fixed
// summation order), diagonalised by cyclic Jacobi in the parallel round-robin
// order (16 disjoint rotations a round, rotations skipped once
// |g_pq| <= 1e-17 sqrt(g_pp g_qq), at most 30 sweeps), and W is replaced by
// W V_k' for the eigenvectors whose eigenvalues exceed tolH/2, largest first:
// ||H - W' W'^T||_2 <= tolH/2 + tolH/2 = tolH, the tolerance of the blocks.
__global__ void __launch_bounds__(256) k_hankel_truncate(DevPtrs P) {
  Item& itr = P.items[blockIdx.x];
  const Item it = itr;
  const int k = it.k;
  if (k <= 1) return;
  constexpr int K = kRS;                   // padded order (k <= kRS - 1)
  constexpr int kCh = 128;
  __shared__ double A[K][K + 1];
  __shared__ double V[K][K + 1];
  __shared__ double chunk[kCh][K + 1];
  __shared__ double rc[K / 2], rs[K / 2];
  __shared__ int rp[K / 2], rq[K / 2];
  __shared__ int any_rot;
  __shared__ int order[K];
  const int t = threadIdx.x;
  const int64_t nh = it.nh;
  double* W = P.W + it.w0;
  // G = W^T W: thread t owns entries e = t and t + 256 of the k x k upper triangle
  int ea[2], eb[2];
  double acc[2] = {0.0, 0.0};
  for (int h = 0; h < 2; ++h) {
    int e = t + 256 * h, a = 0;
    while (e >= k - a && a < k) { e -= k - a; ++a; }
    ea[h] = a < k ? a : -1;
    eb[h] = a < k ? a + e : -1;
  }
  for (int64_t r0 = 0; r0 < nh; r0 += kCh) {
    const int rows = int(min<int64_t>(kCh, nh - r0));
    for (int e = t; e < kCh * k; e += blockDim.x) {
      const int r = e % kCh, c = e / kCh;
      chunk[r][c] = r < rows ? W[r0 + r + int64_t(c) * nh] : 0.0;
    }
    __syncthreads();
    for (int h = 0; h < 2; ++h)
      if (ea[h] >= 0)
        for (int r = 0; r < kCh; ++r) acc[h] = fma(chunk[r][ea[h]], chunk[r][eb[h]], acc[h]);
    __syncthreads();
  }
  for (int e = t; e < K * K; e += blockDim.x) {
    A[e / K][e % K] = 0.0;
    V[e / K][e % K] = (e / K == e % K) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int h = 0; h < 2; ++h)
    if (ea[h] >= 0) {
      A[ea[h]][eb[h]] = acc[h];
      A[eb[h]][ea[h]] = acc[h];
    }
  __syncthreads();
  // cyclic Jacobi, round-robin pairs: round r pairs (r, K-1) and ((r+i) mod (K-1), (r-i) mod (K-1))
  for (int sweep = 0; sweep < 30; ++sweep) {
    if (t == 0) any_rot = 0;
    __syncthreads();
    for (int round = 0; round < K - 1; ++round) {
      if (t < K / 2) {
        int p, q;
        if (t == 0) { p = round; q = K - 1; }
        else { p = (round + t) % (K - 1); q = (round - t + (K - 1)) % (K - 1); }
        if (p > q) { const int w = p; p = q; q = w; }
        const double apq = A[p][q], app = A[p][p], aqq = A[q][q];
        double c = 1.0, sn = 0.0;
        if (apq != 0.0 && fabs(apq) > 1e-17 * sqrt(fabs(app * aqq))) {
          const double th = (aqq - app) / (2.0 * apq);
          const double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          c = 1.0 / sqrt(tt * tt + 1.0);
          sn = tt * c;
          any_rot = 1;
        }
        rp[t] = p; rq[t] = q; rc[t] = c; rs[t] = sn;
      }
      __syncthreads();
      // rows p, q of A <- J^T A
      for (int e = t; e < (K / 2) * K; e += blockDim.x) {
        const int pr = e / K, j = e % K;
        const int p = rp[pr], q = rq[pr];
        const double c = rc[pr], sn = rs[pr];
        const double ap = A[p][j], aq = A[q][j];
        A[p][j] = c * ap - sn * aq;
        A[q][j] = sn * ap + c * aq;
      }
      __syncthreads();
      // columns p, q of A and of V <- (.) J
      for (int e = t; e < (K / 2) * K * 2; e += blockDim.x) {
        const int which = e / ((K / 2) * K);
        const int f = e % ((K / 2) * K);
        const int pr = f / K, i = f % K;
        const int p = rp[pr], q = rq[pr];
        const double c = rc[pr], sn = rs[pr];
        double (*X)[K + 1] = which ? V : A;
        const double xp = X[i][p], xq = X[i][q];
        X[i][p] = c * xp - sn * xq;
        X[i][q] = sn * xp + c * xq;
      }
      __syncthreads();
    }
    if (!any_rot) break;
    __syncthreads();
  }
  // eigenvalues A[i][i], i < k, in decreasing order (ties by index); keep those above tolH/2
  if (t < k) {
    const double li = A[t][t];
    int pos = 0;
    for (int j = 0; j < k; ++j) {
      const double lj = A[j][j];
      pos += (lj > li || (lj == li && j < t)) ? 1 : 0;
    }
    order[pos] = t;
  }
  __syncthreads();
  int kk = 0;
  for (int j = 0; j < k; ++j) kk += A[j][j] > 0.5 * it.tolH ? 1 : 0;
  // W <- W V(:, order[0 .. kk-1]) row by row (in place: a row's outputs need only that row)
  for (int64_t i = t; i < nh; i += blockDim.x) {
    double row[K];
#pragma unroll
    for (int c = 0; c < K; ++c) row[c] = c < k ? W[i + int64_t(c) * nh] : 0.0;
    for (int c = 0; c < kk; ++c) {
      const int src = order[c];
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < K; ++j) v = fma(row[j], V[j][src], v);
      W[i + int64_t(c) * nh] = v;
    }
  }
  __syncthreads();
  if (t == 0) {
    itr.k = kk;
    itr.r = (it.r > it.k) ? kk + 1 : 0;
    P.diag[4 * blockIdx.x + 3] = kk;
  }
}

// Left/right factors of every off-diagonal block of every level (rows are
// independent): level d, row i in child c1 of its node -> U12 row / V21 row;
// in child c2 -> U21 row / V12 row.  Columns 0..k-1 come from W, column k is
// the rank-one corner, the rest are zero.
__global__ void k_assemble_bases(DevPtrs P, int item) {
  const Item it = P.items[item];
  const int d = blockIdx.y;
  if (d >= it.L) return;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= it.n) return;
  const int leaf = P.rowleaf[it.row0 + i];
  const int64_t j = leaf >> (it.L - d);
  const int side = (leaf >> (it.L - d - 1)) & 1;
  const Node nd = P.nodes[node_index(it, d, j)];
  const int64_t o = nd.start, n1 = nd.size / 2;
  const double* W = P.W + it.w0;
  const int64_t nh = it.nh;
  double* XL = P.XL + it.lvl0 + int64_t(d) * it.n * kRS;
  double* XR = P.XR + it.lvl0 + int64_t(d) * it.n * kRS;
  const double nu = it.nu;
  const double dpi = P.dplus[it.row0 + i], dmi = P.dminus[it.row0 + i];
  const int k = it.k, r = it.r;
  if (side == 0) {
    const int64_t p = i - o;                  // row within c1
    const int64_t hp = n1 - 1 - p;            // reversed Hankel index
    for (int s = 0; s < kRS; ++s) {
      double w = (s < k) ? W[hp + int64_t(s) * nh] : 0.0;
      double xl = (s < k) ? -nu * dmi * w : 0.0;
      double xr = w;
      if (s == k && r > k) {
        xl = (p == n1 - 1) ? -nu * dpi : 0.0;  // corner of A12: -nu d+_{o+n1-1} at (n1-1, 0)
        xr = (p == n1 - 1) ? 1.0 : 0.0;        // corner of A21 pairs with e_{n1-1}
      }
      XL[i + int64_t(s) * it.n] = xl;
      XR[i + int64_t(s) * it.n] = xr;
    }
  } else {
    const int64_t q = i - o - n1;             // row within c2
    for (int s = 0; s < kRS; ++s) {
      double w = (s < k) ? W[q + int64_t(s) * nh] : 0.0;
      double xl = (s < k) ? -nu * dpi * w : 0.0;
      double xr = w;
      if (s == k && r > k) {
        xl = (q == 0) ? -nu * dmi : 0.0;        // corner of A21: -nu d-_{o+n1} at (0, n1-1)
        xr = (q == 0) ? 1.0 : 0.0;              // corner of A12 pairs with e_0
      }
      XL[i + int64_t(s) * it.n] = xl;
      XR[i + int64_t(s) * it.n] = xr;
    }
  }
}

// Dense leaves straight from g: M_ij = s [i=j] + nu (d+_i T_ij + d-_i T_ji),
// T_ab = -g_{a-b+1} for b <= a+1.  Padding rows/columns form an identity.
__global__ void k_assemble_leaves(DevPtrs P, int item, int b) {
  const Item it = P.items[item];
  const int64_t l = blockIdx.x;
  const Node nd = P.nodes[node_index(it, it.L, l)];
  const double* g = P.g + it.g0;
  double* A = P.Aleaf + (it.leaf0 + l) * int64_t(b) * b;
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
    const int i = e % b, j = e / b;
    double v;
    if (i >= nd.size || j >= nd.size) {
      v = (i == j) ? 1.0 : 0.0;
    } else {
      const int64_t gi = it.row0 + nd.start + i;
      double tij = (j <= i + 1) ? -g[i - j + 1] : 0.0;
      double tji = (i <= j + 1) ? -g[j - i + 1] : 0.0;
      v = it.nu * (P.dplus[gi] * tij + P.dminus[gi] * tji);
      if (i == j) v += it.shift;
    }
    A[e] = v;
  }
}

}  // namespace hfde
