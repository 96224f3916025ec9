"""Pins of the 1D CPU oracle against what the paper and mathematics fix.

Each test checks ``oracle.fde1d`` against something other than itself:
library special functions, brute-force assembly from the scheme, exact
rational arithmetic, banded textbook solves, closed-form manufactured
solutions and the paper's stated properties (Sec. 2.2.1, Sec. 3.2, Sec. 3.4.2).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.special as sps

from oracle import fde1d as O
import workloads as W


# ---------------------------------------------------------------- g_k -----
@pytest.mark.parametrize("alpha", [1.1, 1.2, 1.5, 1.8, 1.9])
def test_gl_first_values_and_sign_pattern(alpha):
    """g_0 = 1, g_1 = -alpha, g_0 > g_2 > g_3 > ... > 0 (Sec. 2.2.1)."""
    g = O.gl_weights(alpha, 5000)
    assert g[0] == 1.0 and g[1] == -alpha
    tail = g[2:]
    assert np.all(tail > 0)
    assert g[0] > g[2]
    assert np.all(np.diff(tail) < 0)


@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.8])
def test_gl_matches_binomial_definition(alpha):
    """g_k = (-1)^k binom(alpha, k) (eq. (Grun)), via scipy's binomial."""
    g = O.gl_weights(alpha, 60)
    k = np.arange(61)
    ref = (-1.0) ** k * sps.binom(alpha, k)
    np.testing.assert_allclose(g, ref, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.8])
def test_gl_gamma_closed_form(alpha):
    """g_k = alpha(alpha-1) Gamma(k-alpha) / (Gamma(k+1) Gamma(2-alpha)) for k >= 2
    (proof of Lemma hadamard-product), evaluated with log-gamma."""
    n = 70000
    g = O.gl_weights(alpha, n)
    k = np.array([2, 3, 10, 100, 1000, 10000, 65536])
    ref = alpha * (alpha - 1) * np.exp(sps.gammaln(k - alpha) - sps.gammaln(k + 1)
                                       - sps.gammaln(2 - alpha))
    np.testing.assert_allclose(g[k], ref, rtol=2e-9)


@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.8])
def test_gl_partial_sums(alpha):
    """sum_{k<=K} g_k^(alpha) = g_K^(alpha-1): the generating function (1-z)^alpha
    divided by (1-z).  Hence sum g_k -> 0 and sum_{k>=2} g_k -> alpha - 1."""
    K = 4096
    g = O.gl_weights(alpha, K)
    h = O.gl_weights(alpha - 1.0, K)
    ps = np.cumsum(g)
    np.testing.assert_allclose(ps[[10, 100, 1000, K]], h[[10, 100, 1000, K]],
                               rtol=1e-9, atol=K * 2.2e-16 * 2 * alpha)
    assert abs(ps[-1]) < 1e-2           # slowly -> 0 like K^-alpha
    assert abs(ps[-1]) > 0


@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.8])
def test_gl_asymptotic_decay(alpha):
    """g_k = O(k^{-alpha-1}); precisely g_k k^{alpha+1} -> 1/|Gamma(-alpha)|."""
    k = 200000
    g = O.gl_weights(alpha, k)
    assert g[k] * k ** (alpha + 1) == pytest.approx(1.0 / abs(math.gamma(-alpha)), rel=1e-4)


def test_gl_integer_orders():
    """alpha = 2 gives the second difference (1,-2,1,0,..); alpha = 1 gives (1,-1,0,..)."""
    np.testing.assert_array_equal(O.gl_weights(2.0, 6), [1, -2, 1, 0, 0, 0, 0])
    np.testing.assert_array_equal(O.gl_weights(1.0, 4), [1, -1, 0, 0, 0])


# ---------------------------------------------------------- matrices -----
@pytest.mark.parametrize("alpha,n", [(1.2, 7), (1.5, 33), (1.8, 64), (1.7, 1)])
def test_toeplitz_matches_scheme_sums(alpha, n):
    """eq. (toeplitz_FD)/(system_FD) equal the matrix built term by term from the
    two shifted Grunwald-Letnikov sums of Sec. 2.2.1."""
    rng = np.random.default_rng(1)
    dp = rng.uniform(0.5, 2.0, n)
    dm = rng.uniform(0.5, 2.0, n)
    nu = 37.5
    M = O.fd_matrix(alpha, n, nu, dp, dm, 1.0)
    Mb = O.fd_matrix_from_scheme(alpha, n, nu, dp, dm, 1.0)
    np.testing.assert_allclose(M, Mb, rtol=1e-14, atol=1e-12)


def test_fd_rows_equal_rows_of_the_dense_matrix():
    """Selected rows of M formed without the matrix (for sampled checks at
    large N) equal the rows of the dense fd_matrix bit for bit, including the
    first and last rows and the rows next to them."""
    rng = np.random.default_rng(4)
    for alpha, n in [(1.3, 1), (1.3, 2), (1.7, 57), (1.05, 200)]:
        dp, dm = 1 + rng.random(n), 1 + rng.random(n)
        M = O.fd_matrix(alpha, n, 3.7, dp, dm, shift=0.5)
        rows = sorted({0, 1, n - 2, n - 1, n // 2} & set(range(n)))
        R = O.fd_rows(alpha, n, 3.7, dp, dm, rows, shift=0.5)
        assert np.array_equal(R, M[rows])


def test_lean_matrix_equals_the_dense_matrix():
    """The column-block builder used for the stored N = 65536 trajectories
    gives fd_matrix bit for bit (Fortran order, block edges inside and at the
    ends of the matrix, the limits alpha = 1 and 2), and its dense LU solve
    gives the same solution as the plain one."""
    rng = np.random.default_rng(6)
    for alpha, n, blk in [(1.3, 1, 64), (2.0, 2, 1), (1.0, 9, 4), (1.7, 130, 64), (1.05, 301, 100)]:
        dp, dm = 1 + rng.random(n), 1 + rng.random(n)
        M = O.fd_matrix(alpha, n, 3.7, dp, dm, shift=0.5)
        L = O.fd_matrix_lean(alpha, n, 3.7, dp, dm, shift=0.5, block=blk)
        assert L.flags.f_contiguous and np.array_equal(M, L)
    p = W.var_1d(1.8, n=500)
    b = p.u0 + p.dt * p.f
    x1 = O.DenseSolver(p.alpha, p.n, p.nu, p.d_plus, p.d_minus).solve(b)
    x2 = O.DenseSolver(p.alpha, p.n, p.nu, p.d_plus, p.d_minus, lean=True).solve(b)
    assert np.array_equal(x1, x2)


@pytest.mark.parametrize("alpha", [1.1, 1.5, 1.9])
@pytest.mark.parametrize("shift", [1.0, 0.5])
def test_strict_diagonal_dominance(alpha, shift):
    """M is strictly row diagonally dominant (Sec. 2.2.1), with margin >= shift."""
    n = 300
    x, h = W.grid(n)
    dp, dm = 1 + x * x, 1 + (1 - x) ** 2
    nu = (1 / 64) / h ** alpha
    M = O.fd_matrix(alpha, n, nu, dp, dm, shift)
    d = np.abs(np.diag(M))
    off = np.sum(np.abs(M), axis=1) - d
    margin = d - off
    assert np.all(margin > shift * (1 - 1e-9))


def test_alpha2_is_tridiagonal_heat_matrix():
    """alpha = 2: D+ T + D- T^T = (D+ + D-) tridiag(-1, 2, -1); solve vs banded LAPACK."""
    n = 200
    x, h = W.grid(n)
    dp, dm = 1 + x, 2 - x
    nu = 0.01 / h ** 2
    M = O.fd_matrix(2.0, n, nu, dp, dm, 1.0)
    s = nu * (dp + dm)
    ab = np.zeros((3, n))
    ab[0, 1:] = -s[:-1]
    ab[1, :] = 1 + 2 * s
    ab[2, :-1] = -s[1:]
    b = np.sin(np.pi * x) + x
    u_band = sla.solve_banded((1, 1), ab, b)
    np.testing.assert_allclose(M @ u_band, b, rtol=1e-12, atol=1e-12)
    solver = O.DenseSolver(2.0, n, nu, dp, dm, 1.0)
    np.testing.assert_allclose(solver.solve(b), u_band, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("alpha", [1.2, 1.8])
def test_hankel_of_weights_is_psd(alpha):
    """h_ij = g_{i+j} (i, j >= 1) is positive semidefinite (Lemma hadamard-product)."""
    g = O.gl_weights(alpha, 1000)
    idx = np.arange(1, 301)
    H = g[idx[:, None] + idx[None, :]]
    ev = np.linalg.eigvalsh(H)
    assert ev.min() > -1e-14 * ev.max()


# ------------------------------------------------------- dd residual -----
def test_dd_residual_exact_rational():
    """Double-double residual equals the exact rational residual rounded to FP64."""
    n = 12
    alpha, nu, shift = 1.37, 3.25, 1.0
    rng = np.random.default_rng(5)
    dp = rng.uniform(0.5, 2, n)
    dm = rng.uniform(0.5, 2, n)
    x = rng.standard_normal(n)
    g = O.gl_weights(alpha, n + 1)
    M_rows = []
    # b chosen so that cancellation is severe: b ~ M x computed in FP64
    b = O.fd_matrix(alpha, n, nu, dp, dm, shift) @ x
    r = O.residual_dd(alpha, nu, shift, dp, dm, x, b, g=g)
    F = Fraction
    for i in range(n):
        acc = F(b[i]) - F(shift) * F(x[i])
        sp = sum(F(g[i - j + 1]) * F(x[j]) for j in range(0, min(i + 1, n - 1) + 1))
        sm = sum(F(g[j - i + 1]) * F(x[j]) for j in range(max(i - 1, 0), n))
        acc += F(nu) * (F(dp[i]) * sp + F(dm[i]) * sm)
        M_rows.append(acc)
    exact = np.array([float(v) for v in M_rows])
    scale = np.abs(O.fd_matrix(alpha, n, nu, dp, dm, shift)) @ np.abs(x)
    assert np.all(np.abs(r - exact) <= 4 * 2.2e-16 * np.abs(exact) + 1e-30 * scale + 1e-300)


def test_dd_residual_vs_dense_fp64():
    n = 500
    alpha, nu = 1.6, 1234.5
    x, h = W.grid(n)
    dp, dm = 1 + x * x, 1 + (1 - x) ** 2
    u = np.cos(3 * x)
    b = np.zeros(n)
    r = O.residual_dd(alpha, nu, 1.0, dp, dm, u, b)
    M = O.fd_matrix(alpha, n, nu, dp, dm, 1.0)
    scale = np.abs(M) @ np.abs(u)
    assert np.max(np.abs(r + M @ u) / scale) < 1e-13


# ------------------------------------------------------- time stepping -----
def test_dense_solver_refined_residual():
    prob = W.plain_1d()
    S = O.DenseSolver(prob.alpha, prob.n, prob.nu, prob.d_plus, prob.d_minus)
    b = prob.u0 + prob.dt * prob.f
    u = S.solve(b)
    r = O.residual_dd(prob.alpha, prob.nu, 1.0, prob.d_plus, prob.d_minus, u, b)
    M = O.fd_matrix(prob.alpha, prob.n, prob.nu, prob.d_plus, prob.d_minus)
    # the refined solution is a correctly rounded solution up to a few ulps of |M||u|
    assert np.max(np.abs(r) / (np.abs(M) @ np.abs(u))) < 4e-16


@pytest.mark.parametrize("alpha", [1.3, 1.7])
def test_manufactured_solution_first_order(alpha):
    """The shifted GL + implicit Euler scheme is O(dt) + O(dx) (Sec. 2.2.1):
    refining h and dt together halves the error (observed order 1 +- 0.25)."""
    errs = []
    for n in (63, 127, 255):
        errs.append(O.euler_manufactured(alpha, n, steps=n + 1))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert all(0.75 < o < 1.35 for o in orders), (errs, orders)


# --------------------------------------------------------- rank theory -----
@pytest.mark.parametrize("alpha", [1.2, 1.8])
def test_offdiag_ranks_below_beckermann_bound(alpha):
    """eps-rank of every off-diagonal block of T is <= B(N, eps/2) (Lemma fd-qsrank),
    eps relative to ||T||_2."""
    n, eps = 512, 1e-8
    T = O.toeplitz_T(alpha, n)
    tol = eps * np.linalg.norm(T, 2)
    bound = O.beckermann_bound(n, eps / 2)
    worst = 0
    for r0, r1, c0, c1 in O.hodlr_offdiag_blocks(n, 32):
        worst = max(worst, O.eps_rank(T[r0:r1, c0:c1], tol))
    assert worst <= bound
    assert worst >= 4        # the blocks are genuinely rank structured, not trivial


def test_lower_blocks_are_restrictions_of_top_block():
    """Sec. 3.4.2: every subdiagonal block of T at a lower level is a submatrix of
    the top-level block A21 (Toeplitz structure); A12 has one nonzero."""
    n, alpha = 200, 1.4
    T = O.toeplitz_T(alpha, n)
    n1 = n // 2
    top = T[n1:, :n1]
    assert np.count_nonzero(T[:n1, n1:]) == 1 and T[n1 - 1, n1] == -1.0
    for r0, r1, c0, c1 in O.hodlr_offdiag_blocks(n, 8):
        if r0 > c0:   # lower block, rows [r0,r1) cols [c0,c1), touching the diagonal at r0=c1
            m2, m1 = r1 - r0, c1 - c0
            np.testing.assert_array_equal(T[r0:r1, c0:c1], top[:m2, n1 - m1:])


# ------------------------------------------------ time-dependent coefficients
def test_varying_coefficients_constant_in_time_equal_euler():
    """Coefficients that do not change in time reproduce the one-LU stepper."""
    n = 150
    x, h = W.grid(n)
    p = W.Problem1D(n, 1.6, 1 / 16, 5, h, x, 1 + x * x, 1 + (1 - x) ** 2, W.bump(x), np.cos(3 * x))
    u1 = O.euler_1d(p)
    u2 = O.euler_1d_varying(p, lambda t: (p.d_plus, p.d_minus))
    np.testing.assert_allclose(u2, u1, rtol=1e-15, atol=0)


def test_varying_coefficients_alpha2_eigenmode_closed_form():
    """alpha = 2 with d+ = d- = c(t): M(t) = I + 2 nu c(t) tridiag(-1, 2, -1),
    whose eigenvectors sin(j pi x_i) do not depend on t, so the discrete
    solution from u0 = sin(pi x) is u0 times prod_m 1 / (1 + 2 nu c(t_m) lambda_1)
    with lambda_1 = 4 sin^2(pi h / 2)."""
    n, dt, steps = 127, 0.01, 6
    x, h = W.grid(n)
    v = np.sin(np.pi * x)
    one = np.ones(n)
    p = W.Problem1D(n, 2.0, dt, steps, h, x, one, one, v.copy(), np.zeros(n))
    c = lambda t: 1.0 + 0.5 * math.sin(3.0 * t)
    u = O.euler_1d_varying(p, lambda t: (c(t) * one, c(t) * one))
    lam = 4.0 * math.sin(math.pi * h / 2) ** 2
    fac = np.prod([1.0 / (1.0 + 2.0 * p.nu * c(m * dt) * lam) for m in range(1, steps + 1)])
    np.testing.assert_allclose(u, fac * v, rtol=1e-11, atol=1e-14)
