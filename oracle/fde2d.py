"""CPU oracle for the 2D per-step Sylvester equation (test infrastructure).

TEST INFRASTRUCTURE ONLY; see ``oracle/__init__.py``.

Sec. 4.2 rewrites one implicit-Euler step of the 2D equation as
    A U^{(m+1)} + U^{(m+1)} B^T = U^{(m)} + dt F^{(m+1)}       (eq. (sylv-timestepping))
with A = 1/2 I + nu_x (D1+ T_{a1} + D1- T_{a1}^T) acting along x (rows of U)
and  B = 1/2 I + nu_y (D2+ T_{a2} + D2- T_{a2}^T) acting along y (columns).
(The paper writes F without dt; with dt = 1 as in its experiment the two agree;
the implicit-Euler derivation of Sec. 4 gives dt F.)

Three independent ways to compute the exact step:
* ``kron_solve``: the Kronecker system (I (x) A + B (x) I) vec(U) = vec(C)
  (the relation vec(AXB) = (B^T (x) A) vec(X) of Sec. 4.2), brute force.
* ``sylvester_solve``: Bartels-Stewart (scipy.linalg.solve_sylvester);
  ``SylvesterStepper`` reuses the Schur forms and refines each step once.
* ``eig_solve``: orthogonal diagonalisation when A and B are symmetric
  (constant coefficients): U = Q_A [(Q_A^T C Q_B) / (l_i + m_j)] Q_B^T.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .fde1d import fd_matrix


def sylvester_coefficients(prob, shift=0.5):
    """Dense A (nx x nx) and B (ny x ny) of eq. (sylv-timestepping)."""
    A = fd_matrix(prob.alpha_x, prob.nx, prob.nu_x, prob.dxp, prob.dxm, shift)
    B = fd_matrix(prob.alpha_y, prob.ny, prob.nu_y, prob.dyp, prob.dym, shift)
    return A, B


def kron_solve(A, B, C):
    """Solve A X + X B^T = C through (I (x) A + B (x) I) vec X = vec C (column-major vec)."""
    nx, ny = C.shape
    K = np.kron(np.eye(ny), A) + np.kron(B, np.eye(nx))
    x = np.linalg.solve(K, C.reshape(-1, order="F"))
    return x.reshape((nx, ny), order="F")


def sylvester_solve(A, B, C):
    """Bartels-Stewart for A X + X B^T = C."""
    return sla.solve_sylvester(A, B.T, C)


def eig_solve(A, B, C):
    """Symmetric A, B: diagonalise both and divide entrywise."""
    la, Qa = np.linalg.eigh(A)
    lb, Qb = np.linalg.eigh(B)
    Ct = Qa.T @ C @ Qb
    return Qa @ (Ct / (la[:, None] + lb[None, :])) @ Qb.T


class SylvesterStepper:
    """Exact implicit-Euler steps of eq. (sylv-timestepping), Bartels-Stewart per step
    with the real Schur forms of A and B^T computed once.  Bartels-Stewart is
    backward stable, i.e. exact for matrices perturbed by about u ||A||
    (||A|| ~ dt/h^alpha), which in the smooth modes, where the operator is of
    order one, is an error of about u ||A|| in the solution; ``refine`` steps
    of iterative refinement with the FP64 residual C - A X - X B^T (whose
    rounding spreads over all modes) remove it."""

    def __init__(self, prob, shift=0.5):
        self.A, self.B = sylvester_coefficients(prob, shift)
        self.TA, self.ZA = sla.schur(self.A, output="real")
        self.TB, self.ZB = sla.schur(self.B.T, output="real")
        self.dt = prob.dt

    def solve(self, C):
        """X with A X + X B^T = C, reusing the Schur factors (LAPACK trsyl)."""
        F = self.ZA.T @ C @ self.ZB
        Y, scale, info = sla.lapack.dtrsyl(self.TA, self.TB, F)
        if info < 0:
            raise RuntimeError(f"trsyl failed: {info}")
        return self.ZA @ (Y * (1.0 / scale)) @ self.ZB.T

    def step(self, U, F, refine=1):
        C = U + self.dt * F
        X = self.solve(C)
        for _ in range(refine):
            X = X + self.solve(C - self.A @ X - X @ self.B.T)
        return X


def residual(A, B, X, C):
    """C - A X - X B^T."""
    return C - A @ X - X @ B.T
