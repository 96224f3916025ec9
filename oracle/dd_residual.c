/* Double-double residual of the 1D fractional-diffusion operator.
 *
 * TEST INFRASTRUCTURE ONLY (part of the CPU oracle; never linked into the
 * product library).
 *
 * r = b - (s I + nu (D+ T + D- T^T)) x, with T the lower Hessenberg Toeplitz
 * matrix of eq. (toeplitz_FD): T_ij = -g_{i-j+1} for j <= i+1, else 0.
 * With mass_c != 0 the shift term is s (I + mass_c (S + S^T)), S the shift
 * by one row: the mass matrix of the finite-element scheme (Sec. 2.2.2),
 * 2/3 on the diagonal and 1/6 beside it, is (2/3)(I + (S + S^T)/4).
 *   (T x)_i   = -sum_{j <= i+1} g_{i-j+1} x_j
 *   (T^T x)_i = -sum_{j >= i-1} g_{j-i+1} x_j
 * Every product is split exactly with fma (TwoProd) and every sum is carried
 * in double-double (TwoSum, Knuth), so the returned residual is accurate to
 * about one unit roundoff of |r| plus u^2 |M||x|.  The coefficient products
 * nu*d_i*g_k are themselves carried exactly as double-double values.
 * O(N^2) work, O(N) memory; rows are split over OpenMP threads.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double hi, lo; } dd;

static inline dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double err = (a - (s - bb)) + (b - bb);
  dd r = {s, err};
  return r;
}

static inline dd two_prod(double a, double b) {
  double p = a * b;
  double e = fma(a, b, -p);
  dd r = {p, e};
  return r;
}

static inline dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  double lo = s.lo + a.lo + b.lo;
  return two_sum(s.hi, lo);
}

static inline dd dd_mul_d(dd a, double b) {
  dd p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return two_sum(p.hi, p.lo);
}

/* sum over j of coefficient g[idx(j)] * x_j in double-double */
void dd_fd_residual(int64_t n, double nu, double shift, double mass_c,
                    const double* g, const double* dp, const double* dm,
                    const double* x, const double* b, double* r, int threads) {
#ifdef _OPENMP
  if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
  for (int64_t i = 0; i < n; ++i) {
    dd sp = {0.0, 0.0}, sm = {0.0, 0.0};
    /* (G+ x)_i = sum_{j <= i+1} g_{i-j+1} x_j (0-based same offsets) */
    int64_t jmax = i + 1 < n - 1 ? i + 1 : n - 1;
    for (int64_t j = 0; j <= jmax; ++j) sp = dd_add(sp, two_prod(g[i - j + 1], x[j]));
    /* (G- x)_i = sum_{j >= i-1} g_{j-i+1} x_j */
    int64_t jmin = i - 1 > 0 ? i - 1 : 0;
    for (int64_t j = jmin; j < n; ++j) sm = dd_add(sm, two_prod(g[j - i + 1], x[j]));
    /* M x = s x + nu (d+ T x + d- T^T x) = s x - nu (d+ sp + d- sm) */
    dd t = dd_add(dd_mul_d(sp, dp[i]), dd_mul_d(sm, dm[i]));
    t = dd_mul_d(t, nu);
    dd acc = two_sum(b[i], -shift * x[i]);
    acc.lo += fma(-shift, x[i], shift * x[i]);   /* exact remainder of shift*x */
    if (mass_c != 0.0) {
      /* - s mass_c (x_{i-1} + x_{i+1}); s mass_c is exact for mass_c = 1/4 */
      dd nb = two_sum(i > 0 ? x[i - 1] : 0.0, i + 1 < n ? x[i + 1] : 0.0);
      acc = dd_add(acc, dd_mul_d(nb, -shift * mass_c));
    }
    acc = dd_add(acc, t);                          /* b - s x + nu(...) since T = -G */
    r[i] = acc.hi + acc.lo;
  }
}
