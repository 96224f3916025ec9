// HODLR construction of M = s I + nu (D+ T + D- T^T) (or s E + ..., finite
// elements) on gfx950.
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
//
// Finite elements (Sec. 2.2.2, Sec. 3.4.3): M = s E + nu (D+ T + D- T^T) with
// E the P1 mass matrix / h (tridiagonal) and T built the same way from the
// stiffness generator w.  On the uniform grid the blocks have the same
// Toeplitz structure, so the same construction applies, with two changes:
// the Hankel factored is [w_{p+q+3}] (PSD, while w_2 may be negative), which
// leaves each block's first row to an exact rank-one term, and E's
// off-diagonal sits in the same corner as g_0.
#include "internal.hpp"

namespace hfde {

// Finite-element generator (Sec. 2.2.2, eq. (fe-int)): with hats of height 1
// and unit spacing, <phi_{j+m-1}, d^alpha_+ phi_j> is
//   w_m = (1/Gamma(4-alpha)) sum_{t=-2..2} c_t (m-1+t)_+^p,  p = 3 - alpha,
//   c = (1, -4, 6, -4, 1)
// (the derivative is the second derivative of the fractional integral of
// order 2 - alpha, moved onto phi_i; the hat is a second difference of
// truncated powers).  The five terms cancel to a value smaller by about m^4,
// so away from the diagonal (k = m - 1 >= 8) the fourth difference is summed
// instead as its Taylor series about k: the central fourth difference
// operator is (2 sinh(D/2))^4 = sum_{j even >= 4} (2^(j+1) - 8)/j! D^j, so
//   Delta^4 x^p (k) = k^p sum_{j = 4, 6, ...} (2^(j+1) - 8) (p)_j / (j! k^j),
// whose terms are all positive (the sign of (p)_j is that of (p-2)(p-3)) and
// shrink by about (2/k)^2.  Near the diagonal the direct sum loses at most
// 8^4 to cancellation.  Everything is carried in double-double arithmetic
// (error-free sums and products, Dekker and Knuth), the powers by
// x^p = exp(p log x) with a double-double exponential (argument reduction by
// ln 2 and by 2^10, Taylor series, ten squarings) and one Newton step for the
// logarithm, and 1/Gamma(4-alpha) comes from the host in double-double; each
// weight is rounded to FP64 once, so it is the correctly rounded value except
// in rare near-ties.
// Every function turns off floating-point contraction: an error-free
// transformation computes a rounded product and then its rounding error, and
// fusing that product into a later sum (which the gfx950 backend does even
// when the product has other uses) counts the error twice.
namespace fegen {
struct D {
  double hi, lo;
};
__device__ inline D two_sum(double a, double b) {
  #pragma clang fp contract(off)
  const double s = a + b, bb = s - a;
  return D{s, (a - (s - bb)) + (b - bb)};
}
__device__ inline D fast_sum(double a, double b) {   // |a| >= |b|
  #pragma clang fp contract(off)
  const double s = a + b;
  return D{s, b - (s - a)};
}
__device__ inline D add(D a, D b) {
  #pragma clang fp contract(off)
  D s = two_sum(a.hi, b.hi);
  const D t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_sum(s.hi, s.lo);
}
__device__ inline D mul(D a, D b) {
  #pragma clang fp contract(off)
  const double p = a.hi * b.hi;
  double e = fma(a.hi, b.hi, -p);
  e += a.hi * b.lo + a.lo * b.hi;
  return fast_sum(p, e);
}
__device__ inline D mul_d(D a, double b) {
  #pragma clang fp contract(off)
  const double p = a.hi * b;
  double e = fma(a.hi, b, -p);
  e += a.lo * b;
  return fast_sum(p, e);
}
__device__ inline D div_d(D a, double b) {
  #pragma clang fp contract(off)
  const double q = a.hi / b;
  const double p = q * b, pe = fma(q, b, -p);
  const double r = ((a.hi - p) - pe + a.lo) / b;
  return fast_sum(q, r);
}
__device__ inline D scale2(D a, int e) { return D{ldexp(a.hi, e), ldexp(a.lo, e)}; }

// e^a for |a| < 700
__device__ D exp_dd(D a) {
  #pragma clang fp contract(off)
  const D ln2{6.931471805599452862e-01, 2.319046813846299558e-17};
  const double k = rint(a.hi / ln2.hi);
  D r = scale2(add(a, mul_d(ln2, -k)), -10);      // |r| <= ln2 / 2^11
  D s = r, t = r;                                  // s = e^r - 1
  for (int n = 2; n <= 10; ++n) {
    t = div_d(mul(t, r), double(n));
    s = add(s, t);
  }
  for (int i = 0; i < 10; ++i) s = add(mul_d(s, 2.0), mul(s, s));   // e^(2r) - 1 = 2 s + s^2
  return scale2(add(D{1.0, 0.0}, s), int(k));
}

// log x for x > 0 (one Newton step y + x e^-y - 1 from the FP64 logarithm)
__device__ D log_dd(double x) {
  #pragma clang fp contract(off)
  const double y = log(x);
  const D t = mul_d(exp_dd(D{-y, 0.0}), x);
  return add(D{y, 0.0}, add(t, D{-1.0, 0.0}));
}

__device__ D pow_dd(double x, double p) { return exp_dd(mul_d(log_dd(x), p)); }

// w_m, rounded once; ig = 1/Gamma(4 - alpha)
__device__ double weight(int64_t m, double p, D ig) {
  #pragma clang fp contract(off)
  const int64_t k = m - 1;
  D s{0.0, 0.0};
  if (k < 8) {
    const double c[5] = {1.0, -4.0, 6.0, -4.0, 1.0};
    for (int t = -2; t <= 2; ++t) {
      const int64_t x = k + t;
      if (x > 0) s = add(s, mul_d(pow_dd(double(x), p), c[t + 2]));
    }
  } else {
    const double kd = double(k), k2 = kd * kd;     // exact below 2^26
    // b_j = (p)_j / (j! k^j), starting at j = 4
    D b = mul(mul(two_sum(p, 0.0), two_sum(p, -1.0)), mul(two_sum(p, -2.0), two_sum(p, -3.0)));
    b = div_d(div_d(div_d(b, 24.0), k2), k2);
    D sum{0.0, 0.0};
    for (int j = 4; j <= 80; j += 2) {
      const D term = mul(b, two_sum(ldexp(1.0, j + 1), -8.0));   // (2^(j+1) - 8) b_j
      sum = add(sum, term);
      if (fabs(term.hi) <= 1e-34 * fabs(sum.hi)) break;
      b = mul(b, mul(two_sum(p, -double(j)), two_sum(p, -double(j + 1))));
      b = div_d(div_d(b, double((j + 1) * (j + 2))), k2);
    }
    s = mul(pow_dd(kd, p), sum);
  }
  const D w = mul(s, ig);
  return w.hi + w.lo;
}
}  // namespace fegen

// g_0..g_{n+2} by the product recursion g_{k+1} = g_k (k - alpha)/(k + 1)
// (Sec. 3.4.2), evaluated as a blocked multiplicative scan: each thread
// multiplies its segment's factors, one thread scans the segment products,
// then each thread walks its segment again from its prefix.  Finite-element
// operators take the weights w_m of fegen::weight instead.
__global__ void __launch_bounds__(1024) k_gl_weights(DevPtrs P) {
  const Item it = P.items[blockIdx.x];
  const int64_t cnt = it.n + 3;           // g_0 .. g_{n+2}
  double* g = P.g + it.g0;
  if (it.kind == 1) {
    const double p = 3.0 - it.alpha;             // exact for 1 <= alpha <= 2
    const fegen::D ig{it.fig, it.fig_lo};
    for (int64_t m = threadIdx.x; m < cnt; m += blockDim.x) g[m] = fegen::weight(m, p, ig);
    return;
  }
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
  // the largest diagonal entry, a lower bound of ||M||_2 (-g_1 = alpha for
  // the Grunwald-Letnikov weights)
  const double mlow = it.shift * it.mass + it.nu * (-g[1]) * dsum_max;
  const double tau = eps * mlow;
  const double scale = it.nu * dpm;
  const double tolH = scale > 0.0 ? tau / scale : 1e300;
  const int64_t nh = it.nh;
  double* W = P.W + it.w0;
  double* d = P.T1 + it.lvl0;             // residual diagonal (scratch)
  // Hankel of the blocks: H[p][q] = g_{p+q+h0}, h0 = 2 for the differences;
  // h0 = 3 for finite elements, whose w_2 can be negative (then [w_{p+q+2}]
  // is indefinite) while [w_{p+q+3}] is PSD: the blocks' first row is kept
  // apart as a rank-one term (k_assemble_bases).
  const int h0 = 2 + it.kind;
  for (int64_t p = t0; p < nh; p += nt) d[p] = g[2 * p + h0];
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
      double c = g[q + pv + h0];
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
    itr.r = (scale > 0.0 || it.mc != 0.0) ? k + 1 : 0;
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
  if (it.kind == 1) {
    // Finite elements: W factors [g_{p+q+3}], so rows 1.. of each block use
    // W shifted by one row, and the block's first row (towards the diagonal)
    // is the rank-one column k, whose other factor holds that row exactly:
    //   A21[0][p] = -nu (d+_{r2} g_{hp+2} + d-_{r2} g_0 [hp=0]) + s E_{r2,r2-1} [hp=0],
    //   A12[n1-1][q] = -nu (d-_{r1} g_{q+2} + d+_{r1} g_0 [q=0]) + s E_{r1,r1+1} [q=0],
    // r1 = o+n1-1, r2 = o+n1, hp = n1-1-p.
    const double* g = P.g + it.g0;
    const double se = it.shift * it.mass * it.mc;       // off-diagonal of s E
    if (side == 0) {
      const int64_t p = i - o, hp = n1 - 1 - p;
      const int64_t r2 = it.row0 + o + n1;
      for (int s = 0; s < kRS; ++s) {
        double xl = 0.0, xr = 0.0;
        if (s < k) {
          xl = hp >= 1 ? -nu * dmi * W[hp - 1 + int64_t(s) * nh] : 0.0;    // U12
          xr = W[hp + int64_t(s) * nh];                                      // V21
        } else if (s == k) {
          xl = hp == 0 ? 1.0 : 0.0;
          xr = -nu * P.dplus[r2] * g[hp + 2];
          if (hp == 0) xr += -nu * P.dminus[r2] * g[0] + se;
        }
        XL[i + int64_t(s) * it.n] = xl;
        XR[i + int64_t(s) * it.n] = xr;
      }
    } else {
      const int64_t q = i - o - n1;
      const int64_t r1 = it.row0 + o + n1 - 1;
      for (int s = 0; s < kRS; ++s) {
        double xl = 0.0, xr = 0.0;
        if (s < k) {
          xl = q >= 1 ? -nu * dpi * W[q - 1 + int64_t(s) * nh] : 0.0;      // U21
          xr = W[q + int64_t(s) * nh];                                       // V12
        } else if (s == k) {
          xl = q == 0 ? 1.0 : 0.0;
          xr = -nu * P.dminus[r1] * g[q + 2];
          if (q == 0) xr += -nu * P.dplus[r1] * g[0] + se;
        }
        XL[i + int64_t(s) * it.n] = xl;
        XR[i + int64_t(s) * it.n] = xr;
      }
    }
    return;
  }
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

// Dense leaves straight from g: M_ij = s E_ij + nu (d+_i T_ij + d-_i T_ji),
// T_ab = -g_{a-b+1} for b <= a+1, E = I or the P1 mass matrix / h.  Padding
// rows/columns form an identity.
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
      if (i == j) v += it.shift * it.mass;
      else if (it.mc != 0.0 && (i == j + 1 || j == i + 1)) v += it.shift * it.mass * it.mc;
    }
    A[e] = v;
  }
}

}  // namespace hfde
