"""CPU oracle for the 1D fractional diffusion scheme (test infrastructure).

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct FP64 code written
from the paper's definitions.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path
never does.  It shares no code with the HIP library.

What it computes (all FP64):

* ``gl_weights``: the alternating fractional binomial coefficients
  g_k = (-1)^k binom(alpha, k), by the product recursion of Sec. 3.4.2
  (g_0 = 1, g_{k+1} = g_k (k - alpha)/(k + 1)).
* ``toeplitz_T``: the lower Hessenberg Toeplitz matrix T_{alpha,N} of
  eq. (toeplitz_FD), T_ij = -g_{i-j+1} for j <= i+1, else 0.
* ``fd_matrix``: M = s I + nu (D+ T + D- T^T), nu = dt/h^alpha
  (eq. (system_FD); s = 1 in 1D, s = 1/2 for the 2D Sylvester coefficients of
  eq. (sylv-timestepping)).
* ``fd_matrix_lean``: the same matrix, entry for entry, built column block by
  column block in Fortran order (for N where temporaries would not fit).
* ``fd_rows``: selected rows of the same matrix, formed the same way without
  the whole matrix (for sampled checks at large N).
* ``fd_matrix_from_scheme``: the same matrix assembled term by term from the
  two shifted Grunwald-Letnikov sums of Sec. 2.2.1 (boundary values dropped),
  an independent construction used to pin ``fd_matrix``.
* ``euler_1d``: implicit Euler time stepping M u^(m) = u^(m-1) + dt f
  (eq. (system_FD)) with one dense LU (the coefficients do not depend on
  time) and iterative refinement whose residual is computed in
  double-double arithmetic (``residual_dd``), so the result is the exact
  solution of the FP64 system to ~unit roundoff.
* ``manufactured``: the exact solution u = e^{-t} x^2 (1-x)^2 and the source
  that produces it, from the closed-form Riemann-Liouville derivatives of
  eq. (frac-der) (equal to the Grunwald-Letnikov ones for this u, Sec. 2.1).
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import scipy.linalg as sla

_HERE = os.path.dirname(os.path.abspath(__file__))


# --------------------------------------------------------------------------
# Grunwald-Letnikov weights (Sec. 2.1 eq. (Grun); recursion of Sec. 3.4.2)
# --------------------------------------------------------------------------
def gl_weights(alpha: float, n: int) -> np.ndarray:
    """g_0..g_n with g_0 = 1 and g_{k+1} = g_k (k - alpha)/(k + 1)."""
    g = np.empty(n + 1, dtype=np.float64)
    g[0] = 1.0
    for k in range(n):
        g[k + 1] = g[k] * ((k - alpha) / (k + 1))
    return g


# --------------------------------------------------------------------------
# Matrices of eq. (system_FD) / eq. (toeplitz_FD)
# --------------------------------------------------------------------------
def toeplitz_T(alpha: float, n: int) -> np.ndarray:
    """T_{alpha,N}: first column -g_1..-g_N, first row -g_1, -g_0, 0, ..."""
    g = gl_weights(alpha, n)
    col = -g[1:n + 1]
    row = np.zeros(n)
    row[0] = -g[1]
    if n > 1:
        row[1] = -g[0]
    return sla.toeplitz(col, row)


def fd_matrix(alpha, n, nu, d_plus, d_minus, shift=1.0) -> np.ndarray:
    """M = shift*I + nu*(D+ T + D- T^T), dense FP64."""
    T = toeplitz_T(alpha, n)
    M = nu * (np.asarray(d_plus)[:, None] * T + np.asarray(d_minus)[:, None] * T.T)
    M[np.diag_indices(n)] += shift
    return M


def fd_rows(alpha, n, nu, d_plus, d_minus, rows, shift=1.0, g=None) -> np.ndarray:
    """Rows `rows` of M = shift*I + nu*(D+ T + D- T^T), computed as fd_matrix
    does but without forming M (for large N): row i of T holds -g_{i-j+1}
    for j <= i+1 and row i of T^T holds -g_{j-i+1} for j >= i-1 (0-based)."""
    g = gl_weights(alpha, n) if g is None else g
    j = np.arange(n)
    out = np.zeros((len(rows), n))
    for r, i in enumerate(rows):
        k = i - j + 1
        t_row = np.where(k >= 0, -g[np.clip(k, 0, n)], 0.0)
        kt = j - i + 1
        tt_row = np.where(kt >= 0, -g[np.clip(kt, 0, n)], 0.0)
        out[r] = nu * (d_plus[i] * t_row + d_minus[i] * tt_row)
        out[r, i] += shift
    return out


def fd_matrix_lean(alpha, n, nu, d_plus, d_minus, shift=1.0, g=None, block=512) -> np.ndarray:
    """The matrix of ``fd_matrix``, entry for entry the same expression
    nu*(d+_i T_ij + d-_i T_ji) (+ shift on the diagonal), written column block
    by column block into one Fortran-ordered array, so that at large N (65536:
    34 GB) only the matrix itself is held; LAPACK then factors it in place."""
    g = gl_weights(alpha, n) if g is None else g
    dp = np.asarray(d_plus, float)[:, None]
    dm = np.asarray(d_minus, float)[:, None]
    M = np.empty((n, n), order="F")
    i = np.arange(n)[:, None]
    for c0 in range(0, n, block):
        j = np.arange(c0, min(n, c0 + block))[None, :]
        k = i - j + 1                       # T_ij = -g_{i-j+1} where i-j+1 >= 0
        t = np.where(k >= 0, -g[np.clip(k, 0, n)], 0.0)
        kt = j - i + 1                      # (T^T)_ij = T_ji = -g_{j-i+1}
        tt = np.where(kt >= 0, -g[np.clip(kt, 0, n)], 0.0)
        blk = nu * (dp * t + dm * tt)
        d = np.arange(j.shape[1])
        blk[c0 + d, d] += shift
        M[:, c0:c0 + j.shape[1]] = blk
    return M


def fd_matrix_from_scheme(alpha, n, nu, d_plus, d_minus, shift=1.0) -> np.ndarray:
    """Assemble M from the scheme of Sec. 2.2.1, one sum term at a time.

    Row i (1-based) of the scheme reads
      u_i - nu d+_i sum_{k=0}^{i+1} g_k u_{i-k+1}
          - nu d-_i sum_{k=0}^{N-i+2} g_k u_{i+k-1} = rhs_i,
    with u_0 = u_{N+1} = 0 (absorbing boundary) and no other unknowns.
    Pure Python loops: for small N only.
    """
    g = gl_weights(alpha, n + 2)
    M = np.zeros((n, n))
    for i in range(1, n + 1):
        M[i - 1, i - 1] += shift
        for k in range(0, i + 2):
            j = i - k + 1
            if 1 <= j <= n:
                M[i - 1, j - 1] -= nu * d_plus[i - 1] * g[k]
        for k in range(0, n - i + 3):
            j = i + k - 1
            if 1 <= j <= n:
                M[i - 1, j - 1] -= nu * d_minus[i - 1] * g[k]
    return M


# --------------------------------------------------------------------------
# Double-double residual r = b - M x, straight from g (no stored matrix)
# --------------------------------------------------------------------------
_dd_lib = None


def _load_dd():
    global _dd_lib
    if _dd_lib is None:
        path = os.path.join(_HERE, "libdd_residual.so")
        if not os.path.exists(path):
            build_c()
        lib = ctypes.CDLL(path)
        lib.dd_fd_residual.restype = None
        lib.dd_fd_residual.argtypes = [
            ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        _dd_lib = lib
    return _dd_lib


def build_c() -> str:
    """Compile the oracle's C helper (double-double residual) with gcc."""
    src = os.path.join(_HERE, "dd_residual.c")
    out = os.path.join(_HERE, "libdd_residual.so")
    import subprocess
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared",
                           "-fPIC", src, "-o", out + ".tmp", "-lm"])
    os.replace(out + ".tmp", out)
    return out


def residual_dd(alpha, nu, shift, d_plus, d_minus, x, b, g=None, threads=0, mass_c=0.0):
    """r = b - (shift I + nu (D+ T + D- T^T)) x in double-double, rounded to FP64.

    Every product nu*d_i*g_k is formed exactly (TwoProd) and every sum is
    carried in double-double, so the result is the residual of the operator
    whose entries are nu*d*g to ~unit roundoff of r (not of |M||x|).
    With mass_c != 0 the shift term is shift*(I + mass_c*(S + S^T)) (the
    finite-element mass matrix, see ``oracle.fe``).
    """
    n = x.size
    if g is None:
        g = gl_weights(alpha, n + 1)
    lib = _load_dd()
    x = np.ascontiguousarray(x, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    dp = np.ascontiguousarray(d_plus, dtype=np.float64)
    dm = np.ascontiguousarray(d_minus, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    r = np.empty(n)
    lib.dd_fd_residual(n, float(nu), float(shift), float(mass_c), g.ctypes.data, dp.ctypes.data,
                       dm.ctypes.data, x.ctypes.data, b.ctypes.data, r.ctypes.data,
                       int(threads))
    return r


def matvec_dense(alpha, nu, shift, d_plus, d_minus, x):
    """Plain M @ x with a dense matrix (small N)."""
    return fd_matrix(alpha, x.size, nu, d_plus, d_minus, shift) @ x


# --------------------------------------------------------------------------
# Implicit Euler time stepping (eq. (system_FD))
# --------------------------------------------------------------------------
class DenseSolver:
    """Dense LU of M once (LAPACK getrf), solves with double-double refinement."""

    def __init__(self, alpha, n, nu, d_plus, d_minus, shift=1.0, refine=3, lean=False):
        self.alpha, self.n, self.nu, self.shift = alpha, n, nu, shift
        self.d_plus = np.asarray(d_plus, float)
        self.d_minus = np.asarray(d_minus, float)
        self.g = gl_weights(alpha, n + 1)
        if lean:   # same matrix, built without temporaries (large N)
            M = fd_matrix_lean(alpha, n, nu, d_plus, d_minus, shift, g=self.g)
        else:
            M = fd_matrix(alpha, n, nu, d_plus, d_minus, shift)
        self.lu = sla.lu_factor(M, overwrite_a=True, check_finite=False)
        self.refine = refine

    def solve(self, b, refine=None):
        refine = self.refine if refine is None else refine
        x = sla.lu_solve(self.lu, b, check_finite=False)
        for _ in range(refine):
            r = residual_dd(self.alpha, self.nu, self.shift, self.d_plus, self.d_minus,
                            x, b, g=self.g)
            x = x + sla.lu_solve(self.lu, r, check_finite=False)
        return x


def euler_1d(prob, steps=None, refine=3, keep_all=False):
    """u^(m) = M^{-1}(u^(m-1) + dt f), m = 1..steps (f time independent)."""
    steps = prob.steps if steps is None else steps
    S = DenseSolver(prob.alpha, prob.n, prob.nu, prob.d_plus, prob.d_minus, 1.0, refine)
    u = prob.u0.copy()
    out = []
    for _ in range(steps):
        u = S.solve(u + prob.dt * prob.f)
        if keep_all:
            out.append(u.copy())
    return (u, out) if keep_all else u


def euler_1d_varying(prob, coef, steps=None, refine=3):
    """Implicit Euler with coefficients that change in time: at step m the
    matrix of eq. (system_FD) is built from d+(x, t_m), d-(x, t_m) (the new
    time level, t_m = m dt), so every step has its own dense LU:
    u^(m) = M(t_m)^{-1}(u^(m-1) + dt f).  coef(t) -> (d_plus, d_minus)."""
    steps = prob.steps if steps is None else steps
    u = prob.u0.copy()
    for m in range(1, steps + 1):
        dp, dm = coef(m * prob.dt)
        u = DenseSolver(prob.alpha, prob.n, prob.nu, dp, dm, 1.0, refine).solve(u + prob.dt * prob.f)
    return u


# --------------------------------------------------------------------------
# Manufactured solution (eq. (frac-der) closed forms)
# --------------------------------------------------------------------------
def rl_power_derivative(p: float, alpha: float, z: np.ndarray) -> np.ndarray:
    """Left RL derivative of order alpha of z^p: Gamma(p+1)/Gamma(p+1-alpha) z^(p-alpha)."""
    return math.gamma(p + 1) / math.gamma(p + 1 - alpha) * z ** (p - alpha)


def manufactured(alpha, x, t, d_plus, d_minus):
    """u = e^{-t} x^2 (1-x)^2 on [0,1] and f = u_t - d+ D+^a u - d- D-^a u."""
    u = math.exp(-t) * x * x * (1 - x) ** 2
    lap_p = np.zeros_like(x)
    lap_m = np.zeros_like(x)
    for p, c in ((2, 1.0), (3, -2.0), (4, 1.0)):
        lap_p += c * rl_power_derivative(p, alpha, x)
        lap_m += c * rl_power_derivative(p, alpha, 1.0 - x)
    f = -u - math.exp(-t) * (d_plus * lap_p + d_minus * lap_m)
    return u, f


def euler_manufactured(alpha, n, steps, d_fun=lambda x: np.ones_like(x)):
    """Run the scheme on the manufactured problem to T=1; return max-norm error at T."""
    h = 1.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    dt = 1.0 / steps
    dp = d_fun(x)
    dm = d_fun(x)
    nu = dt / h ** alpha
    M = fd_matrix(alpha, n, nu, dp, dm, 1.0)
    lu = sla.lu_factor(M)
    u, _ = manufactured(alpha, x, 0.0, dp, dm)
    for m in range(1, steps + 1):
        _, f = manufactured(alpha, x, m * dt, dp, dm)
        u = sla.lu_solve(lu, u + dt * f)
    ue, _ = manufactured(alpha, x, 1.0, dp, dm)
    return np.max(np.abs(u - ue))


# --------------------------------------------------------------------------
# Rank-structure helpers (Sec. 3; used by structure tests)
# --------------------------------------------------------------------------
def beckermann_bound(n: int, eps: float) -> int:
    """B(N, eps) = 2 + 2 ceil((2/pi^2) log(4N/pi) log(16/eps)) (Lemma beckermann)."""
    return 2 + 2 * math.ceil((2 / math.pi ** 2) * math.log(4 * n / math.pi)
                             * math.log(16 / eps))


def eps_rank(A: np.ndarray, tol_abs: float) -> int:
    """Number of singular values of A above tol_abs."""
    s = np.linalg.svd(A, compute_uv=False)
    return int(np.sum(s > tol_abs))


def hodlr_offdiag_blocks(n: int, leaf: int):
    """(row0, row1, col0, col1) of every off-diagonal block of the 2x2 recursive
    partition of Sec. 3.4.1 (N1 = floor(n/2), N2 = ceil(n/2)), split while n > leaf."""
    out = []

    def rec(o, m):
        if m <= leaf:
            return
        m1 = m // 2
        out.append((o + m1, o + m, o, o + m1))      # lower block A21
        out.append((o, o + m1, o + m1, o + m))      # upper block A12
        rec(o, m1)
        rec(o + m1, m - m1)

    rec(0, n)
    return out
