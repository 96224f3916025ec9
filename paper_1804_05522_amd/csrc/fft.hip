// Exact matrix-vector product with M = s I + nu (D+ T + D- T^T) (eq. (system_FD))
// for the refinement residual, on gfx950.
//
// Sec. 3.4.2 applies T with the FFT (circulant embedding).  Here T is split
//   T = T_near + T_far,  T_near = entries with -1 <= i-j <= w (band),
//                        T_far  = entries with i-j > w  (the slowly decaying tail),
// T_near x and T_near^T x are summed directly in double-double (TwoSum /
// TwoProd with fma), and only the far tail goes through a circulant of
// length M >= 2N-1 (power of two):
//   c[k] = -g_{k+1} for w < k < N, 0 elsewhere,  lambda = FFT(c),
//   T_far x = Re IFFT(mu . FFT(x)),  T_far^T x = Im IFFT(mu . FFT(x)),
//   mu = lambda + i conj(lambda)
// (C^T is the circulant with eigenvalues conj(lambda) because c is real, and
// both products are real, so one complex inverse transform returns both).
// The far tail is small (|g_k| ~ k^{-alpha-1}), so the FFT's rounding error
// is scaled down by the same factor, and the residual is accurate to a few
// units of roundoff of |r| plus a far smaller FFT term.
//
// FFT: radix-2 in LDS after a bit-reversed load (lengths <= 8192); longer
// lengths use the four-step split M = M1 * M2 (two LDS passes with a twiddle
// multiply between them), each pass moving tiles of T adjacent sub-transforms
// so global accesses stay 256-byte contiguous.
#include "internal.hpp"

namespace hfde {

constexpr int kFftWG = 512;
constexpr int kFft4WG = 512;         // threads of a four-step pass work-group
constexpr int kFftLds = 8192;          // complex values held in LDS


__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// In-place radix-2 DIT on `ntile` transforms of length m = 2^logm stored
// back to back in LDS (already in bit-reversed order).  tw: the M-th roots
// e^{-2 pi i j / M} of the problem, M = 2^logM >= m.
__device__ void lds_fft(double2* buf, int ntile, int logm, const double2* tw, int logM, bool inverse) {
  const int m = 1 << logm;
  const int half_total = ntile * (m >> 1);
  for (int lh = 0; lh < logm; ++lh) {
    const int h = 1 << lh;
    const int shift = logM - lh - 1;          // w = omega_{2h}^k = tw[k << shift]
    for (int b = threadIdx.x; b < half_total; b += blockDim.x) {
      const int t = b >> (logm - 1);
      const int q = b & ((m >> 1) - 1);
      const int k = q & (h - 1);
      const int i0 = t * m + ((q >> lh) << (lh + 1)) + k;
      const int i1 = i0 + h;
      double2 w = tw[int64_t(k) << shift];
      if (inverse) w = cconj(w);
      const double2 a = buf[i0];
      const double2 c = cmul(buf[i1], w);
      buf[i0] = make_double2(a.x + c.x, a.y + c.y);
      buf[i1] = make_double2(a.x - c.x, a.y - c.y);
    }
    __syncthreads();
  }
}

__device__ inline int bitrev(int v, int logm) {
  return logm == 0 ? 0 : int(__brev(uint32_t(v)) >> (32 - logm));
}

// --------------------------------------------------------- double-double
// Each function below turns off floating-point contraction: an error-free
// transformation computes a rounded product and then its rounding error, and
// fusing that product into a later sum (which the gfx950 backend does even
// when the product has other uses) counts the error twice.
struct dd {
  double hi, lo;
};
__device__ inline dd two_sum(double a, double b) {
  #pragma clang fp contract(off)
  double s = a + b;
  double bb = s - a;
  return dd{s, (a - (s - bb)) + (b - bb)};
}
__device__ inline dd dd_add(dd a, dd b) {
  #pragma clang fp contract(off)
  dd s = two_sum(a.hi, b.hi);
  return two_sum(s.hi, s.lo + a.lo + b.lo);
}
__device__ inline dd dd_prod(double a, double b) {
  #pragma clang fp contract(off)
  double p = a * b;
  return dd{p, fma(a, b, -p)};
}
__device__ inline dd dd_mul_d(dd a, double b) {
  #pragma clang fp contract(off)
  dd p = dd_prod(a.hi, b);
  p.lo += a.lo * b;
  return two_sum(p.hi, p.lo);
}

// Output of the exact product for row i: y_i = s (E x)_i + nu (d+ (Tn x + far_re) + d- (Tn^T x + far_im)),
// or the residual b_i - y_i (E = I, or the P1 mass matrix / h).  Near band in double-double.
// Chain q (terms k = q - 1 + 4t) of the compensated near-band sums of row i:
//   (T x)_i = -sum_{j <= i+1} g_{i-j+1} x_j ;  near: i - j in [-1, w]
//   (T^T x)_i = -sum_{j >= i-1} g_{j-i+1} x_j ;  near: j - i in [-1, w]
// Compensated dot products (Ogita, Rump and Oishi, "Accurate sum and dot
// product", 2005, algorithm Dot2): the running sum advances by error-free
// additions and the rounding errors of the sums and products collect in a
// second double, which gives the accuracy of twice the working precision.
// Each sum runs in four interleaved chains (terms k = q mod 4) that are
// combined in double-double at the end; rows whose whole band lies inside
// the problem skip the range checks.
struct NearChain {
  double ps, pc, ms, mc;
};

// xat(k) reads x[i + k] (through the LDS window of x); gat(k) reads g_k.
template <typename XA, typename GA>
__device__ inline NearChain exact_chain_t(XA xat, GA gat, int64_t i, int64_t n, int w, int q) {
  NearChain c{0.0, 0.0, 0.0, 0.0};
  auto acc = [](double& sum, double& err, double a, double b) {
    #pragma clang fp contract(off)
    const double p = a * b;
    const double e = fma(a, b, -p);
    const dd t = two_sum(sum, p);
    sum = t.hi;
    err += t.lo + e;
  };
  if (i - w >= 0 && i + w < n && i + 1 < n && i >= 1) {
    for (int k = q - 1; k <= w; k += 4) {
      const double gk = -gat(k + 1);
      acc(c.ps, c.pc, gk, xat(-k));
      acc(c.ms, c.mc, gk, xat(k));
    }
  } else {
    for (int k = q - 1; k <= w; k += 4) {
      const double gk = -gat(k + 1);
      if (i - k >= 0 && i - k < n) acc(c.ps, c.pc, gk, xat(-k));
      if (i + k >= 0 && i + k < n) acc(c.ms, c.mc, gk, xat(k));
    }
  }
  return c;
}

// Row i of M x (or of b - M x) from its four near chains and the far-field
// values left by the inverse transform.
__device__ inline double exact_finish(const DevPtrs& P, const Item& it, const double* x, int64_t i, const NearChain* c,
                                      double far_re, double far_im, const double* bvec) {
  #pragma clang fp contract(off)
  dd sp = dd_add(dd_add(two_sum(c[0].ps, c[0].pc), two_sum(c[1].ps, c[1].pc)),
                 dd_add(two_sum(c[2].ps, c[2].pc), two_sum(c[3].ps, c[3].pc)));
  dd sm = dd_add(dd_add(two_sum(c[0].ms, c[0].mc), two_sum(c[1].ms, c[1].mc)),
                 dd_add(two_sum(c[2].ms, c[2].mc), two_sum(c[3].ms, c[3].mc)));
  sp = dd_add(sp, dd{far_re, 0.0});
  sm = dd_add(sm, dd{far_im, 0.0});
  const int64_t gi = it.row0 + i;
  dd tsum = dd_add(dd_mul_d(sp, P.dplus[gi]), dd_mul_d(sm, P.dminus[gi]));
  tsum = dd_mul_d(tsum, it.nu);
  const double se = it.shift * it.mass;
  dd y = dd_add(dd_prod(se, x[i]), tsum);
  if (it.mc != 0.0) {   // finite elements: s E x = s (2/3)(x_i + (x_{i-1} + x_{i+1})/4)
    const dd nb = two_sum(i > 0 ? x[i - 1] : 0.0, i + 1 < it.n ? x[i + 1] : 0.0);
    y = dd_add(y, dd_mul_d(nb, se * it.mc));
  }
  if (bvec != nullptr) {
    dd r = dd_add(dd{bvec[i], 0.0}, dd{-y.hi, -y.lo});
    return r.hi + r.lo;
  }
  return y.hi + y.lo;
}

// ---------------------------------------------------------------- setup
__global__ void k_twiddles(DevPtrs P, int item) {
  const Item it = P.items[item];
  const int64_t M = int64_t(1) << it.fftlog;
  double2* tw = P.tw + it.tw0;
  for (int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < M; j += int64_t(gridDim.x) * blockDim.x) {
    // e^{-2 pi i j/M}: the argument 2j/M is exact in binary
    double s, c;
    sincospi(-2.0 * double(j) / double(M), &s, &c);
    tw[j] = make_double2(c, s);
  }
}

// value of the far circulant's first column at position k (length M)
__device__ inline double cfar(const DevPtrs& P, const Item& it, int64_t k) {
  if (k > it.band && k < it.n) return -P.g[it.g0 + k + 1];
  return 0.0;
}

// modes of the FFT kernels
enum { kModeSetup = 0, kModeMatvec = 1 };

// Single work-group path (M <= kFftLds): setup builds mu, matvec does the
// whole product for one (problem, column).
__global__ void __launch_bounds__(kFftWG) k_fft_small(DevPtrs P, const FftUnit* units, int mode, const double* x,
                                                     int64_t ldx, double* y, int64_t ldy, const double* b,
                                                     int64_t ldb) {
  extern __shared__ double2 buf[];
  const FftUnit u = units[blockIdx.x];
  const Item it = P.items[u.item];
  const int logM = it.fftlog;
  const int M = 1 << logM;
  const double2* tw = P.tw + it.tw0;
  const double* xc = x ? x + it.row0 + int64_t(u.col) * ldx : nullptr;
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    double v = 0.0;
    if (mode == kModeSetup) v = cfar(P, it, j);
    else if (j < it.n) v = xc[j];
    buf[bitrev(j, logM)] = make_double2(v, 0.0);
  }
  __syncthreads();
  lds_fft(buf, 1, logM, tw, logM, false);
  double2* mu = P.mu + it.mu0;
  if (mode == kModeSetup) {
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
      const double2 l = buf[j];
      mu[j] = make_double2(l.x + l.y, l.y + l.x);   // lambda + i conj(lambda)
    }
    return;
  }
  // multiply, store bit-reversed for the inverse pass
  __syncthreads();
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    const double2 v = cmul(buf[j], mu[j]);
    buf[j] = v;
  }
  __syncthreads();
  // bit-reverse permutation in place (swap pairs once)
  for (int j = threadIdx.x; j < M; j += blockDim.x) {
    const int r = bitrev(j, logM);
    if (r > j) {
      const double2 a = buf[j];
      buf[j] = buf[r];
      buf[r] = a;
    }
  }
  __syncthreads();
  lds_fft(buf, 1, logM, tw, logM, true);
  // far-field values for k_exact_rows, which adds the near band (second half
  // of the column's scratch, where the four-step path leaves them too)
  const double inv = 1.0 / double(M);
  double2* far = P.fws + fws_off(P, it, u.col) + M;
  for (int64_t i = threadIdx.x; i < it.n; i += blockDim.x) {
    const double2 w = buf[i];
    far[i] = make_double2(w.x * inv, w.y * inv);
  }
  (void)y; (void)ldy; (void)b; (void)ldb;
}

// As lds_fft, with the m/2 roots e^{-2 pi i j / m} of the transform length
// staged in LDS (tws), so that no stage waits on global memory.
constexpr int kTwLds = 1024;           // roots held in LDS (transforms up to 2048 points)
__device__ void lds_fft_tw(double2* buf, int ntile, int logm, const double2* twsp, bool inverse) {
  const int m = 1 << logm;
  const ldsd* tws = lds_view(reinterpret_cast<const double*>(twsp));   // re, im interleaved
  ldsd* b3 = lds_view(reinterpret_cast<double*>(buf));
  const double sgn = inverse ? -1.0 : 1.0;
  // (x, y) <- (x + w y, x - w y), w = tws[j] (conjugated for the inverse)
  auto bfly = [&](double& xr, double& xi, double& yr, double& yi, int j) {
    const double wr = tws[2 * j], wi = sgn * tws[2 * j + 1];
    const double cr = yr * wr - yi * wi, ci = yr * wi + yi * wr;
    yr = xr - cr;
    yi = xi - ci;
    xr = xr + cr;
    xi = xi + ci;
  };
  int lh = 0;
  // stages lh and lh + 1 together: one thread takes the four elements
  // k, k + h, k + 2h, k + 3h of a block of 4h (the same butterflies as two
  // radix-2 stages, half the barriers)
  for (; lh + 1 < logm; lh += 2) {
    const int h = 1 << lh;
    const int quarter_total = ntile * (m >> 2);
    for (int b = threadIdx.x; b < quarter_total; b += blockDim.x) {
      const int t = b >> (logm - 2);
      const int q = b & ((m >> 2) - 1);
      const int k = q & (h - 1);
      const int i0 = t * m + ((q >> lh) << (lh + 2)) + k;
      double r0 = b3[2 * i0], j0 = b3[2 * i0 + 1];
      double r1 = b3[2 * (i0 + h)], j1 = b3[2 * (i0 + h) + 1];
      double r2 = b3[2 * (i0 + 2 * h)], j2 = b3[2 * (i0 + 2 * h) + 1];
      double r3 = b3[2 * (i0 + 3 * h)], j3 = b3[2 * (i0 + 3 * h) + 1];
      bfly(r0, j0, r1, j1, k << (logm - lh - 1));            // stage lh, span h
      bfly(r2, j2, r3, j3, k << (logm - lh - 1));
      bfly(r0, j0, r2, j2, k << (logm - lh - 2));            // stage lh + 1, span 2h
      bfly(r1, j1, r3, j3, (k + h) << (logm - lh - 2));
      b3[2 * i0] = r0;
      b3[2 * i0 + 1] = j0;
      b3[2 * (i0 + h)] = r1;
      b3[2 * (i0 + h) + 1] = j1;
      b3[2 * (i0 + 2 * h)] = r2;
      b3[2 * (i0 + 2 * h) + 1] = j2;
      b3[2 * (i0 + 3 * h)] = r3;
      b3[2 * (i0 + 3 * h) + 1] = j3;
    }
    __syncthreads();
  }
  if (lh < logm) {                            // a last radix-2 stage
    const int h = 1 << lh;
    const int half_total = ntile * (m >> 1);
    for (int b = threadIdx.x; b < half_total; b += blockDim.x) {
      const int t = b >> (logm - 1);
      const int q = b & ((m >> 1) - 1);
      const int k = q & (h - 1);
      const int i0 = t * m + ((q >> lh) << (lh + 1)) + k;
      const int i1 = i0 + h;
      double r0 = b3[2 * i0], j0 = b3[2 * i0 + 1], r1 = b3[2 * i1], j1 = b3[2 * i1 + 1];
      bfly(r0, j0, r1, j1, k << (logm - lh - 1));
      b3[2 * i0] = r0;
      b3[2 * i0 + 1] = j0;
      b3[2 * i1] = r1;
      b3[2 * i1 + 1] = j1;
    }
    __syncthreads();
  }
}

// Transform of `ntile` tiles of length 2^logm in buf: with the roots staged
// in LDS when they fit, else read from the problem's root table.
__device__ inline void tile_fft(double2* buf, double2* tws, int ntile, int logm, const double2* tw, int logM,
                                bool inverse) {
  if ((1 << logm) / 2 <= kTwLds) lds_fft_tw(buf, ntile, logm, tws, inverse);
  else lds_fft(buf, ntile, logm, tw, logM, inverse);
}

// Four-step split: M = M1 * M2, n = n1 + M1 n2, k = k2 + M2 k1.
// Columns per work-group of a four-step pass: fewer columns give more
// work-groups per pass (the passes are latency-bound at these lengths), more
// give longer contiguous segments (tile x 16 bytes).
constexpr int kFftTileMax = 2;

__device__ inline void four_step_dims(int logM, int& l1, int& l2, int& tile) {
  l2 = logM / 2;
  l1 = logM - l2;
  tile = kFftLds >> l1;
  if (tile > kFftTileMax) tile = kFftTileMax;
}

// Pass 1: transforms over n2 (length M2) for `tile` adjacent n1, then the
// twiddle omega_M^{n1 k2}; output Y[k2 * M1 + n1].
// forward/setup: input c (setup) or x (matvec, real); inverse: input W.
__global__ void __launch_bounds__(kFft4WG) k_fft4_pass1(DevPtrs P, const FftUnit* units, int mode, bool inverse,
                                                      const double* x, int64_t ldx) {
  extern __shared__ double2 buf[];
  const FftUnit u = units[blockIdx.x];
  const Item it = P.items[u.item];
  const int logM = it.fftlog;
  int l1, l2, T;
  four_step_dims(logM, l1, l2, T);
  const int M1 = 1 << l1, M2 = 1 << l2;
  const double2* tw = P.tw + it.tw0;
  double2* ws = P.fws + fws_off(P, it, u.col);
  double2* Y = ws;                               // first half: Y
  const double2* Win = ws + (int64_t(1) << logM);   // second half: W (inverse input)
  const int n1base = u.tile * T;
  const double* xc = x ? x + it.row0 + int64_t(u.col) * ldx : nullptr;
  __shared__ double2 tws[kTwLds];
  if (M2 / 2 <= kTwLds)
    for (int j = threadIdx.x; j < M2 / 2; j += blockDim.x) tws[j] = tw[int64_t(j) << (logM - l2)];
  for (int e = threadIdx.x; e < T * M2; e += blockDim.x) {
    const int t = e % T, n2 = e / T;
    const int64_t nidx = int64_t(n1base + t) + int64_t(M1) * n2;
    double2 v;
    if (inverse) {
      v = Win[nidx];
    } else if (mode == kModeSetup) {
      v = make_double2(cfar(P, it, nidx), 0.0);
    } else {
      v = make_double2(nidx < it.n ? xc[nidx] : 0.0, 0.0);
    }
    buf[t * M2 + bitrev(n2, l2)] = v;
  }
  __syncthreads();
  tile_fft(buf, tws, T, l2, tw, logM, inverse);
  const int64_t Mmask = (int64_t(1) << logM) - 1;
  for (int e = threadIdx.x; e < T * M2; e += blockDim.x) {
    const int t = e % T, k2 = e / T;
    const int n1 = n1base + t;
    double2 w = tw[(int64_t(n1) * k2) & Mmask];
    if (inverse) w = cconj(w);
    Y[int64_t(k2) * M1 + n1] = cmul(buf[t * M2 + k2], w);
  }
}

// Pass 2: transforms over n1 (length M1) for `tile` adjacent k2; output index
// k = k2 + M2 k1.  setup: mu; forward matvec: W = mu . X (second half of the
// scratch); inverse: the far-field products (scaled by 1/M) in natural order
// into the second half of the scratch, for k_exact_rows.  Every output goes to
// the half the pass does not read: an output index k lies in rows of Y that
// other work-groups of the same launch read.
__global__ void __launch_bounds__(kFft4WG) k_fft4_pass2(DevPtrs P, const FftUnit* units, int mode, bool inverse,
                                                      const double* x, int64_t ldx, double* y, int64_t ldy,
                                                      const double* b, int64_t ldb) {
  extern __shared__ double2 buf[];
  const FftUnit u = units[blockIdx.x];
  const Item it = P.items[u.item];
  const int logM = it.fftlog;
  int l1, l2, T;
  four_step_dims(logM, l1, l2, T);
  const int M1 = 1 << l1, M2 = 1 << l2;
  const int64_t M = int64_t(1) << logM;
  const double2* tw = P.tw + it.tw0;
  double2* ws = P.fws + fws_off(P, it, u.col);
  const double2* Y = ws;
  double2* Wout = ws + M;
  const int k2base = u.tile * T;
  __shared__ double2 tws[kTwLds];
  if (M1 / 2 <= kTwLds)
    for (int j = threadIdx.x; j < M1 / 2; j += blockDim.x) tws[j] = tw[int64_t(j) << (logM - l1)];
  for (int e = threadIdx.x; e < T * M1; e += blockDim.x) {
    const int n1 = e % M1, t = e / M1;
    buf[t * M1 + bitrev(n1, l1)] = Y[int64_t(k2base + t) * M1 + n1];
  }
  __syncthreads();
  tile_fft(buf, tws, T, l1, tw, logM, inverse);
  double2* mu = P.mu + it.mu0;
  const double inv = 1.0 / double(M);
  const double* xc = x ? x + it.row0 + int64_t(u.col) * ldx : nullptr;
  double* yc = y ? y + it.row0 + int64_t(u.col) * ldy : nullptr;
  const double* bc = b ? b + it.row0 + int64_t(u.col) * ldb : nullptr;
  for (int e = threadIdx.x; e < T * M1; e += blockDim.x) {
    const int t = e % T, k1 = e / T;
    const int64_t k = int64_t(k2base + t) + int64_t(M2) * k1;
    const double2 v = buf[t * M1 + k1];
    if (mode == kModeSetup) {
      mu[k] = make_double2(v.x + v.y, v.y + v.x);
    } else if (!inverse) {
      Wout[k] = cmul(v, mu[k]);
    } else if (k < it.n) {
      Wout[k] = make_double2(v.x * inv, v.y * inv);
    }
  }
  (void)xc; (void)yc; (void)bc;
}

// Near-field rows (double-double) plus the far-field values left by the
// inverse pass 2: four lanes per row, one per near chain (the chains are
// independent, so the row's sums have four times the lanes to hide their
// latency), gathered in the row's first lane, which finishes the row.  A unit
// is 256 rows; the work-group has 1024 threads.
constexpr int kExactRowsWG = 1024;
__global__ void __launch_bounds__(kExactRowsWG) k_exact_rows(DevPtrs P, const FftUnit* units, const double* x,
                                                             int64_t ldx, double* y, int64_t ldy, const double* b,
                                                             int64_t ldb) {
  constexpr int kRows = kExactRowsWG / 4, kPad = 66;     // the band is at most 64 wide
  __shared__ double xs[kRows + 2 * kPad];
  __shared__ double gs[kPad + 2];
  const FftUnit u = units[blockIdx.x];
  const Item it = P.items[u.item];
  const int q = threadIdx.x & 3, lane = threadIdx.x & 63;
  const int64_t i0 = int64_t(u.tile) * kRows;
  const int64_t i = i0 + (threadIdx.x >> 2);
  const bool valid = i < it.n;
  const double* xc = x + it.row0 + int64_t(u.col) * ldx;
  // the tile's rows of x with the band on both sides, and the weights, in LDS
  for (int e = threadIdx.x; e < kRows + 2 * kPad; e += blockDim.x) {
    const int64_t j = i0 - kPad + e;
    xs[e] = (j >= 0 && j < it.n) ? xc[j] : 0.0;
  }
  const double* g = P.g + it.g0;
  for (int e = threadIdx.x; e < it.band + 2; e += blockDim.x) gs[e] = g[e];
  __syncthreads();
  const ldsd* xw = lds_view(xs) + (kPad + (threadIdx.x >> 2));    // x[i] of this row
  const ldsd* gw = lds_view(gs);
  const NearChain mine =
      valid ? exact_chain_t([&](int k) { return xw[k]; }, [&](int k) { return gw[k]; }, i, it.n, it.band, q)
            : NearChain{0.0, 0.0, 0.0, 0.0};
  NearChain c[4];
#pragma unroll
  for (int s2 = 0; s2 < 4; ++s2) {
    const int src = (lane & ~3) + s2;
    c[s2].ps = __shfl(mine.ps, src);
    c[s2].pc = __shfl(mine.pc, src);
    c[s2].ms = __shfl(mine.ms, src);
    c[s2].mc = __shfl(mine.mc, src);
  }
  if (q != 0 || !valid) return;
  const int64_t M = int64_t(1) << it.fftlog;
  const double2 w = P.fws[fws_off(P, it, u.col) + M + i];   // far field
  const double* bc = b ? b + it.row0 + int64_t(u.col) * ldb : nullptr;
  y[it.row0 + int64_t(u.col) * ldy + i] = exact_finish(P, it, xc, i, c, w.x, w.y, bc);
}

}  // namespace hfde
