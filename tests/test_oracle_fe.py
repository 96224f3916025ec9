"""Pins of the finite-element oracle (oracle/fe.py) against what the
mathematics fixes: the stiffness entries of eq. (fe-int) by an independent
quadrature route, the reflection K- = K+^T, the limits alpha = 2 (the P1
Laplacian) and alpha = 1 (the P1 convection matrix), the zero sum of a
derivative of a constant, the positive semidefinite Hankel tail that the
compression relies on (Sec. 3.4.3), coercivity, second-order convergence on a
manufactured steady problem, the double-double residual with the mass term,
and the 2D step of eq. (sylv-timestepping-fe) against the Kronecker system."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fde1d
from oracle import fe


@pytest.mark.parametrize("alpha", [1.3, 1.7])
def test_weights_match_quadrature(alpha):
    """w_{k+1} = <phi_{j+k}, d^alpha_+ phi_j> (unit spacing), the integral of
    eq. (fe-int) taken by quadrature of the closed-form derivative of phi_j."""
    w = fe.fe_weights(alpha, 40)
    for k in (-1, 0, 1, 2, 3, 7, 20):
        q = fe.fe_entry_quadrature(alpha, 40 + k, 40, "+")
        assert abs(w[k + 1] - q) <= 1e-9 * max(abs(q), 1e-3), (k, w[k + 1], q)
    # entries above the first superdiagonal vanish: the supports do not meet
    assert fe.fe_entry_quadrature(alpha, 38, 40, "+") == 0.0


@pytest.mark.parametrize("alpha", [1.3, 1.7])
def test_right_derivative_is_transpose(alpha):
    """K-_ij = <phi_i, d^alpha_- phi_j> = w_{j-i+1} = K+_ji."""
    w = fe.fe_weights(alpha, 40)
    for k in (-1, 0, 1, 2, 5):
        q = fe.fe_entry_quadrature(alpha, 40, 40 + k, "-")
        assert abs(w[k + 1] - q) <= 1e-9 * max(abs(q), 1e-3), (k, w[k + 1], q)


def test_integer_order_limits():
    """alpha = 2: the P1 matrix of u'' (1, -2, 1), which equals the
    Grunwald-Letnikov generator at alpha = 2; alpha = 1: the P1 matrix of u'
    (<phi_i, phi_{i+1}'> = 1/2, <phi_i, phi_{i-1}'> = -1/2)."""
    w2 = fe.fe_weights(2.0, 12)
    assert np.allclose(w2, [1, -2, 1] + [0] * 9, atol=1e-15)
    assert np.allclose(w2, fde1d.gl_weights(2.0, 11), atol=1e-15)
    w1 = fe.fe_weights(1.0, 12)
    assert np.allclose(w1, [0.5, 0, -0.5] + [0] * 9, atol=1e-15)
    # and the 2D-free consequence: at alpha = 2 the finite-element matrix is
    # the finite-difference one plus the mass matrix in place of the identity
    n, nu = 30, 0.7
    d = np.linspace(1.0, 2.0, n)
    A = fe.fe_matrix(2.0, n, nu, d, d[::-1], 1.0)
    B = fde1d.fd_matrix(2.0, n, nu, d, d[::-1], 0.0) + fe.mass_matrix(n)
    assert np.allclose(A, B, rtol=0, atol=1e-14)


@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.8])
def test_weights_sum_to_zero(alpha):
    """The hats sum to 1 away from the boundary and the derivative of a
    constant on a half line vanishes, so sum_m w_m = 0; the partial sums decay
    like m^(-alpha) (the tail of w_m ~ m^(-1-alpha))."""
    w = fe.fe_weights(alpha, 4097)
    s1, s2 = abs(w[:2049].sum()), abs(w[:4097].sum())
    assert s2 < s1 < 1e-3
    assert abs(math.log2(s1 / s2) - alpha) < 0.05
    # signs: w_0 > 0, w_1 < 0, w_m > 0 from m = 3 on
    assert w[0] > 0 and w[1] < 0 and np.all(w[3:] > 0)


@pytest.mark.parametrize("alpha", [1.1, 1.3, 1.5, 1.7, 1.9])
def test_hankel_tail_is_psd(alpha):
    """[w_{p+q+3}] is positive semidefinite (for m >= 3 every point of the
    fourth difference lies in x >= 0, where x^(3-alpha) is a mixture of
    exponentials, so w_m is a moment sequence): the factorisation the
    construction uses.  [w_{p+q+2}] is not PSD in general (w_2 < 0 at
    alpha = 1.3), which is why the first row of each block is kept apart."""
    w = fe.fe_weights(alpha, 500)
    n = 200
    H3 = np.array([[w[p + q + 3] for q in range(n)] for p in range(n)])
    ev = np.linalg.eigvalsh(H3)
    assert ev.min() >= -1e-14 * ev.max()
    if alpha == 1.3:
        assert w[2] < 0


@pytest.mark.parametrize("alpha", [1.3, 1.7])
def test_stiffness_is_coercive(alpha):
    """-(K + K^T) is positive semidefinite: the real parts of the spectrum of
    the pencil (A, E) lie at or right of the shift."""
    n = 200
    T = fe.fe_matrix(alpha, n, 1.0, np.ones(n), np.zeros(n), 0.0)   # T itself (D+ = I, no mass)
    ev = np.linalg.eigvalsh(T + T.T)
    assert ev.min() >= -1e-12


def test_mass_matrix():
    """<phi_i, phi_i> = 2h/3, <phi_i, phi_{i+1}> = h/6: rows sum to 1."""
    E = fe.mass_matrix(8)
    assert np.allclose(E[1:-1].sum(axis=1), 1.0)
    v = np.random.default_rng(0).standard_normal((8, 3))
    assert np.allclose(fe.mass_apply(v), E @ v, atol=1e-15)


def _steady_error(alpha, n):
    """Max nodal error of the P1 Galerkin solution of -(d+ + d-)-derivative
    problem -(D+^a u + D-^a u) = f with u = x^2 (1-x)^2 on [0, 1]."""
    h = 1.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    T = fe.fe_matrix(alpha, n, 1.0, np.ones(n), np.ones(n), 0.0)    # = -(W + W^T)
    K = -h ** (1 - alpha) * T                                        # K+ + K-

    def f(z):
        s = 0.0
        for p, c in ((2, 1.0), (3, -2.0), (4, 1.0)):
            s = s + c * (fde1d.rl_power_derivative(p, alpha, z) + fde1d.rl_power_derivative(p, alpha, 1 - z))
        return -s

    gx, gw = np.polynomial.legendre.leggauss(20)
    load = np.zeros(n)
    for e in range(n + 1):
        z = e * h + h * (gx + 1) / 2
        t = (gx + 1) / 2
        fz = f(z) * gw * h / 2
        if e >= 1:
            load[e - 1] += np.sum(fz * (1 - t))
        if e < n:
            load[e] += np.sum(fz * t)
    u = np.linalg.solve(-K, load)
    return np.max(np.abs(u - x * x * (1 - x) ** 2))


@pytest.mark.parametrize("alpha", [1.3, 1.7])
def test_manufactured_steady_second_order(alpha):
    """The Galerkin solution converges at second order at the nodes: a wrong
    scale (Gamma factor, power of h), sign or transposition breaks it."""
    e = [_steady_error(alpha, n) for n in (31, 63, 127)]
    rates = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert e[0] < 2e-4 and min(rates) > 1.8, (e, rates)


def test_residual_dd_with_mass():
    """The double-double residual with the mass term equals b - A x formed
    with the dense matrix (to the dense product's rounding)."""
    rng = np.random.default_rng(1)
    n = 300
    dp, dm = 1 + rng.random(n), 1 + rng.random(n)
    x, b = rng.standard_normal(n), rng.standard_normal(n)
    A = fe.fe_matrix(1.4, n, 37.0, dp, dm, 0.5)
    r = fe.residual_dd(1.4, 37.0, 0.5, dp, dm, x, b)
    ref = b - A @ x
    assert np.max(np.abs(r - ref)) <= 1e-13 * np.max(np.abs(A) @ np.abs(x))


def test_time_step():
    """One step of the 1D scheme: (E + nu (...)) u1 = E (u0 + dt f)."""
    p = W.fe_1d(n=200, steps=1)
    u1 = fe.euler_fe_1d(p, steps=1)
    A = fe.fe_matrix(p.alpha, p.n, p.nu, p.d_plus, p.d_minus, 1.0)
    ref = np.linalg.solve(A, fe.mass_matrix(p.n) @ (p.u0 + p.dt * p.f))
    assert np.max(np.abs(u1 - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_2d_step_against_kronecker():
    """The paper's route (mass matrices inverted, then Bartels-Stewart) equals
    the brute-force Kronecker solve of the generalized equation."""
    p = W.fe_2d(n=14)
    st = fe.FeSylvesterStepper(p)
    U0, F = p.u0.dense(), p.f.dense()
    X = st.step(U0, F)
    Xk = fe.fe_kron_solve(st.A, st.B, st.Ex, st.Ey, st.rhs(U0, F))
    assert np.max(np.abs(X - Xk)) <= 1e-12 * np.max(np.abs(Xk))
    R = fe.generalized_residual(st.A, st.B, st.Ex, st.Ey, X, st.rhs(U0, F))
    assert np.linalg.norm(R) <= 1e-13 * np.linalg.norm(st.rhs(U0, F))


def test_2d_step_refinement():
    """At a size where the Kronecker system is still solvable (n = 40), the
    refined step is closer to the Kronecker solution than the plain
    Bartels-Stewart step, and within a few u of it."""
    p = W.fe_2d(n=40)
    st = fe.FeSylvesterStepper(p)
    U0, F = p.u0.dense(), p.f.dense()
    Xk = fe.fe_kron_solve(st.A, st.B, st.Ex, st.Ey, st.rhs(U0, F))
    e0 = np.linalg.norm(st.step(U0, F, refine=0) - Xk)
    e1 = np.linalg.norm(st.step(U0, F, refine=1) - Xk)
    assert e1 <= e0 and e1 <= 1e-14 * np.linalg.norm(Xk), (e0, e1)
