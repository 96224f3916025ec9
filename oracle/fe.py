"""CPU oracle for the finite-element discretisation (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Plain, slow FP64 code written from the paper's
finite-element scheme (Sec. 2.2.2, Sec. 3.4.3, eq. (sylv-timestepping-fe));
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the product path never does.  It shares no code
with the HIP library.

Discretisation.  Hat functions phi_1..phi_N of height 1 on the uniform grid
x_i = L + i h (support [x_{i-1}, x_{i+1}]), the stiffness matrices
(K+-)_ij = <phi_i, d^alpha_+- phi_j> with the Riemann-Liouville derivatives of
eq. (frac-der), and the mass matrix (M)_ij = <phi_i, phi_j>.  Implicit Euler
(Sec. 2.2.2):  (M - dt (D+ K+ + D- K-)) u^(m) = M u^(m-1) + dt M f, where the
load <f, phi_i> is taken for the P1 interpolant of f.

What it computes:

* ``fe_weights``: the generator w of the stiffness, K+_ij = h^(1-alpha)
  w_{i-j+1}.  Derivation: for 1 < alpha < 2 the left derivative is the second
  derivative of the fractional integral of order 2 - alpha; moving both
  derivatives onto phi_i (whose second derivative is (delta_{x_{i-1}} -
  2 delta_{x_i} + delta_{x_{i+1}})/h) and writing the hat as a second
  difference of truncated powers (x - c)_+, whose fractional integral of
  order beta is (x - c)_+^(1+beta) / Gamma(2+beta), gives
      w_m = (1/Gamma(4-alpha)) sum_{t=-2..2} c_t (m - 1 + t)_+^(3-alpha),
      c = (1, -4, 6, -4, 1)
  (a fourth difference).  Far from the diagonal the five terms cancel to a
  value smaller by about m^4 (the numerical instability the paper notes in
  Sec. (ex-fe)), so each w_m is evaluated in mpmath with enough digits and
  rounded once.  K+ is lower Hessenberg (for i - j + 1 < 0 the support of
  phi_i lies left of that of d^alpha_+ phi_j) and K- = K+^T by reflection.
* ``fe_entry_quadrature``: one entry <phi_i, d^alpha_+- phi_j> by adaptive
  quadrature of phi_i times the closed-form derivative of phi_j (an
  independent route: one integration by parts fewer).
* ``mass_matrix``: M / h = tridiag(1/6, 2/3, 1/6).
* ``fe_matrix``: s E + nu (D+ T + D- T^T) with E = M/h, T_ij = -w_{i-j+1}
  and nu = dt / h^alpha: the Galerkin matrix s M - dt (D+ K+ + D- K-)
  divided by h.  With variable coefficients d+-(x) are sampled at the test
  function's node (a row scaling); for constant coefficients, the paper's
  finite-element experiment, this is the Galerkin matrix itself.
* ``FeSolver``, ``euler_fe_1d``: dense LU time stepping with
  double-double-residual refinement.
* ``fe_sylvester_coefficients``, ``FeSylvesterStepper``: the 2D step of
  eq. (sylv-timestepping-fe), A U E_y + E_x U B^T = E_x (U_prev + dt F) E_y
  with A = 1/2 E_x + nu_x (...), solved as the paper does in its experiment:
  E_x^{-1} and E_y^{-1} applied first, then Bartels-Stewart on
  (E_x^{-1} A) U + U (E_y^{-1} B)^T = U_prev + dt F, plus one step of
  iterative refinement on the generalized equation.
* ``fe_kron_solve``: the same step through the Kronecker system
  (E_y (x) A + B (x) E_x) vec U = vec C (brute force, tiny sizes).
"""
from __future__ import annotations

import math

import mpmath
import numpy as np
import scipy.linalg as sla

from . import fde1d

_FOURTH = (1, -4, 6, -4, 1)
_W_CACHE: dict = {}


def fe_weights(alpha: float, count: int) -> np.ndarray:
    """w_0 .. w_{count-1} of the P1 stiffness generator, each rounded once
    from a multi-precision evaluation of the fourth difference."""
    key = (float(alpha), int(count))
    if key in _W_CACHE:
        return _W_CACHE[key].copy()
    # the five terms are about m^(3-alpha), the result about m^(-1-alpha):
    # m^4 is lost to cancellation, so carry 25 digits beyond that
    digits = 25 + int(4 * math.log10(max(count, 10)) + 1)
    w = np.empty(count)
    with mpmath.workdps(digits):
        p = mpmath.mpf(3) - mpmath.mpf(alpha)
        ig = 1 / mpmath.gamma(4 - mpmath.mpf(alpha))
        pw = {}

        def tp(x):
            if x <= 0:
                return mpmath.mpf(0)
            if x not in pw:
                pw[x] = mpmath.power(x, p)
            return pw[x]

        for m in range(count):
            s = mpmath.mpf(0)
            for t, c in zip(range(-2, 3), _FOURTH):
                s += c * tp(m - 1 + t)
            w[m] = float(s * ig)
            pw.pop(m - 3, None)
    _W_CACHE[key] = w.copy()
    return w


def fe_entry_quadrature(alpha: float, i: int, j: int, side: str = "+") -> float:
    """<phi_i, d^alpha_side phi_j> for unit spacing (h = 1, nodes at the
    integers, supports away from the boundary), by mpmath quadrature split at
    the nodes.  The left derivative of the hat is
        (1/Gamma(2-alpha)) sum_m c_m (x - (j+m))_+^(1-alpha), c = (1, -2, 1);
    the right one mirrors it."""
    a = mpmath.mpf(alpha)
    ig = 1 / mpmath.gamma(2 - a)

    def dphi(x):
        s = mpmath.mpf(0)
        for m, c in ((-1, 1), (0, -2), (1, 1)):
            z = (x - (j + m)) if side == "+" else ((j + m) - x)
            if z > 0:
                s += c * mpmath.power(z, 1 - a)
        return s * ig

    def phi(x):
        return max(mpmath.mpf(0), 1 - abs(x - i))

    pts = sorted({i - 1, i, i + 1} | {j + m for m in (-1, 0, 1) if i - 1 < j + m < i + 1})
    with mpmath.workdps(30):
        v = mpmath.quad(lambda x: phi(x) * dphi(x), pts, maxdegree=10)
    return float(v)


def mass_matrix(n: int) -> np.ndarray:
    """E = M/h: 2/3 on the diagonal, 1/6 beside it."""
    E = np.zeros((n, n))
    E[np.diag_indices(n)] = 2.0 / 3.0
    i = np.arange(n - 1)
    E[i, i + 1] = 1.0 / 6.0
    E[i + 1, i] = 1.0 / 6.0
    return E


def mass_apply(v: np.ndarray) -> np.ndarray:
    """E v along the first axis (zero outside the grid)."""
    out = (2.0 / 3.0) * v
    out[1:] += (1.0 / 6.0) * v[:-1]
    out[:-1] += (1.0 / 6.0) * v[1:]
    return out


def fe_matrix(alpha, n, nu, d_plus, d_minus, shift=1.0, w=None) -> np.ndarray:
    """s E + nu (D+ T + D- T^T), T_ij = -w_{i-j+1} (j <= i+1), dense FP64."""
    w = fe_weights(alpha, n + 1) if w is None else w
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    k = i - j + 1
    T = np.where(k >= 0, -w[np.clip(k, 0, n)], 0.0)
    M = nu * (np.asarray(d_plus, float)[:, None] * T + np.asarray(d_minus, float)[:, None] * T.T)
    return M + shift * mass_matrix(n)


def residual_dd(alpha, nu, shift, d_plus, d_minus, x, b, w=None, threads=0):
    """r = b - (s E + nu (D+ T + D- T^T)) x in double-double (the oracle's C
    helper with the mass term: s E x = (s 2/3)(x_i + (x_{i-1} + x_{i+1})/4))."""
    n = x.size
    w = fe_weights(alpha, n + 1) if w is None else w
    return fde1d.residual_dd(alpha, nu, shift * (2.0 / 3.0), d_plus, d_minus, x, b, g=w,
                             threads=threads, mass_c=0.25)


class FeSolver:
    """Dense LU of the finite-element matrix, solves refined with the
    double-double residual."""

    def __init__(self, alpha, n, nu, d_plus, d_minus, shift=1.0, refine=3):
        self.alpha, self.n, self.nu, self.shift = alpha, n, nu, shift
        self.d_plus = np.asarray(d_plus, float)
        self.d_minus = np.asarray(d_minus, float)
        self.w = fe_weights(alpha, n + 1)
        self.lu = sla.lu_factor(fe_matrix(alpha, n, nu, d_plus, d_minus, shift, w=self.w),
                                overwrite_a=True, check_finite=False)
        self.refine = refine

    def solve(self, b, refine=None):
        refine = self.refine if refine is None else refine
        x = sla.lu_solve(self.lu, b, check_finite=False)
        for _ in range(refine):
            r = residual_dd(self.alpha, self.nu, self.shift, self.d_plus, self.d_minus, x, b, w=self.w)
            x = x + sla.lu_solve(self.lu, r, check_finite=False)
        return x


def euler_fe_1d(prob, steps=None, refine=3, keep_all=False):
    """(E + nu (D+ T + D- T^T)) u^(m) = E (u^(m-1) + dt f), m = 1..steps."""
    steps = prob.steps if steps is None else steps
    S = FeSolver(prob.alpha, prob.n, prob.nu, prob.d_plus, prob.d_minus, 1.0, refine)
    u = prob.u0.copy()
    out = []
    for _ in range(steps):
        u = S.solve(mass_apply(u + prob.dt * prob.f))
        if keep_all:
            out.append(u.copy())
    return (u, out) if keep_all else u


# --------------------------------------------------------------------------
# 2D: eq. (sylv-timestepping-fe)
# --------------------------------------------------------------------------
def fe_sylvester_coefficients(prob, shift=0.5):
    """Dense A, B (shift E + nu (...)) and the mass matrices E_x, E_y."""
    A = fe_matrix(prob.alpha_x, prob.nx, prob.nu_x, prob.dxp, prob.dxm, shift)
    B = fe_matrix(prob.alpha_y, prob.ny, prob.nu_y, prob.dyp, prob.dym, shift)
    return A, B, mass_matrix(prob.nx), mass_matrix(prob.ny)


def fe_kron_solve(A, B, Ex, Ey, C):
    """A X E_y + E_x X B^T = C through (E_y (x) A + B (x) E_x) vec X = vec C."""
    nx, ny = C.shape
    K = np.kron(Ey, A) + np.kron(B, Ex)
    return np.linalg.solve(K, C.reshape(-1, order="F")).reshape((nx, ny), order="F")


def generalized_residual(A, B, Ex, Ey, X, C):
    """C - A X E_y - E_x X B^T."""
    return C - A @ X @ Ey - Ex @ X @ B.T


def _mass_solve(v: np.ndarray) -> np.ndarray:
    """E^{-1} v along the first axis (tridiagonal solve)."""
    n = v.shape[0]
    ab = np.zeros((3, n))
    ab[0, 1:] = 1.0 / 6.0
    ab[1, :] = 2.0 / 3.0
    ab[2, :-1] = 1.0 / 6.0
    return sla.solve_banded((1, 1), ab, v)


class FeSylvesterStepper:
    """Exact implicit-Euler steps of eq. (sylv-timestepping-fe), by the
    paper's route for its experiment: the mass matrices are inverted first,
    so each step is the Sylvester equation
        (E_x^{-1} A) U + U (E_y^{-1} B)^T = U_prev + dt F,
    solved by Bartels-Stewart with the real Schur forms computed once.
    Bartels-Stewart is backward stable for the reduced matrices, whose norm
    is that of the stiffness (about dt/h^alpha), so its solution carries
    errors of about u ||A|| in the smooth modes, where the operator is of
    order one; ``refine`` steps of iterative refinement with the residual of
    the generalized equation itself (formed in FP64; its rounding spreads
    over all modes) remove them."""

    def __init__(self, prob, shift=0.5):
        self.A, self.B, self.Ex, self.Ey = fe_sylvester_coefficients(prob, shift)
        At = sla.solve(self.Ex, self.A)
        Bt = sla.solve(self.Ey, self.B)
        self.TA, self.ZA = sla.schur(At, output="real")
        self.TB, self.ZB = sla.schur(Bt.T, output="real")
        self.dt = prob.dt

    def solve_reduced(self, Ct):
        F = self.ZA.T @ Ct @ self.ZB
        Y, scale, info = sla.lapack.dtrsyl(self.TA, self.TB, F)
        if info < 0:
            raise RuntimeError(f"trsyl failed: {info}")
        return self.ZA @ (Y * (1.0 / scale)) @ self.ZB.T

    def step(self, U, F, refine=1):
        X = self.solve_reduced(U + self.dt * F)
        C = self.rhs(U, F)
        for _ in range(refine):
            R = C - mass_apply((self.A @ X).T).T - mass_apply(X @ self.B.T)
            X = X + self.solve_reduced(_mass_solve(_mass_solve(R).T).T)
        return X

    def rhs(self, U, F):
        """The right-hand side of the generalized equation, E_x (U + dt F) E_y."""
        return self.Ex @ (U + self.dt * F) @ self.Ey
