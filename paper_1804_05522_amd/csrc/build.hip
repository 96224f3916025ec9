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
    if (vsum <= tolH || vmax <= 0.0) break;
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
