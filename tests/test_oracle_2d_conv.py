"""Pins of the 2D Sylvester oracle and of the conv-net oracle."""
import numpy as np
import pytest
import scipy.signal as ssig

from oracle import fde1d as O1
from oracle import fde2d as O2
from oracle import convnet as C
import workloads as W


def _small2d(n=24, variable=True):
    p = W.fd_2d(n=n, variable=variable, dt=1 / 8)
    return p


def test_vec_kronecker_identity():
    """vec(A X B) = (B^T (x) A) vec(X) (Sec. 4.2), column-major vec."""
    rng = np.random.default_rng(0)
    A, X, B = rng.standard_normal((5, 5)), rng.standard_normal((5, 4)), rng.standard_normal((4, 4))
    lhs = (A @ X @ B).reshape(-1, order="F")
    rhs = np.kron(B.T, A) @ X.reshape(-1, order="F")
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("variable", [False, True])
def test_sylvester_solvers_agree(variable):
    p = _small2d(24, variable)
    A, B = O2.sylvester_coefficients(p)
    rng = np.random.default_rng(2)
    Cm = rng.standard_normal((p.nx, p.ny))
    Xk = O2.kron_solve(A, B, Cm)
    Xs = O2.sylvester_solve(A, B, Cm)
    st = O2.SylvesterStepper(p)
    Xt = st.solve(Cm)
    np.testing.assert_allclose(Xs, Xk, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(Xt, Xk, rtol=1e-10, atol=1e-12)
    if not variable:
        Xe = O2.eig_solve(A, B, Cm)
        np.testing.assert_allclose(Xe, Xk, rtol=1e-10, atol=1e-12)


def test_2d_step_equals_kron_implicit_euler():
    """One step of eq. (sylv-timestepping) is the implicit Euler step of the 2D
    operator (I + nu_x L_x (x) ... ) assembled from the 1D matrices with shift 1."""
    p = _small2d(16, True)
    Ax = O1.fd_matrix(p.alpha_x, p.nx, p.nu_x, p.dxp, p.dxm, 0.0)
    By = O1.fd_matrix(p.alpha_y, p.ny, p.nu_y, p.dyp, p.dym, 0.0)
    K = np.eye(p.nx * p.ny) + np.kron(np.eye(p.ny), Ax) + np.kron(By, np.eye(p.nx))
    U0 = np.outer(np.sin(np.pi * p.x), p.y * (1 - p.y))
    F = p.f.dense()
    u1 = np.linalg.solve(K, (U0 + p.dt * F).reshape(-1, order="F")).reshape(U0.shape, order="F")
    st = O2.SylvesterStepper(p)
    np.testing.assert_allclose(st.step(U0, F), u1, rtol=1e-11, atol=1e-13)


def test_2d_step_refinement():
    """At n = 40 (Kronecker system still solvable) the refined step is at
    least as close to the Kronecker solution as the plain Bartels-Stewart
    step, and within a few u of it (the 4096^2 golden step uses it)."""
    p = W.fd_2d(n=40, dt=0.1)
    st = O2.SylvesterStepper(p)
    rng = np.random.default_rng(5)
    U0 = rng.standard_normal((40, 3)) @ rng.standard_normal((3, 40))
    F = p.f.dense()
    Xk = O2.kron_solve(st.A, st.B, U0 + p.dt * F)
    e0 = np.linalg.norm(st.step(U0, F, refine=0) - Xk)
    e1 = np.linalg.norm(st.step(U0, F, refine=1) - Xk)
    assert e1 <= e0 and e1 <= 1e-14 * np.linalg.norm(Xk), (e0, e1)


# ------------------------------------------------------------- convnet -----
def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 3, 9, 7))
    w = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    y = C.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(ssig.correlate2d(x[n, c], w[o, c], mode="same", boundary="fill")
                             for c in range(3))
            np.testing.assert_allclose(y[n, o], ref, rtol=1e-12, atol=1e-12)


def test_convnet_gradients_finite_differences():
    rng = np.random.default_rng(4)
    params = C.init_params(rng, channels=4, scale_last=1.0)
    u = rng.standard_normal((2, 1, 6, 5))
    tgt = rng.standard_normal((2, 1, 6, 5))
    loss, grads = C.loss_and_grads(params, u, tgt)
    h = 1e-6
    for li in range(4):
        for k in range(2):
            arr = params[li][k]
            flat = arr.reshape(-1)
            for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp, _ = C.loss_and_grads(params, u, tgt)
                flat[idx] = old - h
                lm, _ = C.loss_and_grads(params, u, tgt)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                an = grads[li][k].reshape(-1)[idx]
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (li, k, idx, fd, an)


def test_adam_first_step_is_signed_lr():
    """With zero moments, Adam's first update is lr * g/(|g| + eps) ~ lr sign(g)."""
    params = [[np.array([1.0, -2.0, 3.0]), np.zeros(1)]]
    grads = [[np.array([0.5, -4.0, 1e-3]), np.array([2.0])]]
    opt = C.Adam(params, lr=0.1)
    opt.step(params, grads)
    np.testing.assert_allclose(params[0][0], [0.9, -1.9, 2.9], rtol=1e-6)
    np.testing.assert_allclose(params[0][1], [-0.1], rtol=1e-6)


def test_adam_constant_gradient_every_step():
    """A constant gradient g makes both bias-corrected moments exact at every
    step (mhat = g, vhat = g^2), so each of five steps moves every parameter by
    exactly lr g/(|g| + eps).  A bias correction evaluated at t = 1, or the two
    decay rates exchanged, breaks this from the second step on."""
    g = np.array([0.5, -4.0, 1e-3, 7.0])
    lr, eps = 0.05, 1e-8
    params = [[np.array([1.0, -2.0, 3.0, 0.0])]]
    opt = C.Adam(params, lr=lr, eps=eps)
    for t in range(1, 6):
        before = params[0][0].copy()
        opt.step(params, [[g.copy()]])
        np.testing.assert_allclose(before - params[0][0], lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)


def test_adam_alternating_gradient_closed_form():
    """Gradients +g, -g, +g, ... : the moments have the geometric-series closed
    forms m_t = (1-b1) g (-1)^(t+1) (1 - (-b1)^t)/(1 + b1) and v_t = g^2 (1 - b2^t),
    so vhat = g^2 exactly and mhat = m_t/(1 - b1^t); the parameter after t steps
    is the sum of the resulting updates.  Checked for t = 1..8 against the
    recurrence of the optimiser."""
    b1, b2, lr, eps = 0.9, 0.999, 0.01, 1e-8
    g = np.array([2.0, -0.25])
    p0 = np.array([0.3, 0.7])
    params = [[p0.copy()]]
    opt = C.Adam(params, lr=lr, b1=b1, b2=b2, eps=eps)
    expect = p0.copy()
    for t in range(1, 9):
        sgn = 1.0 if t % 2 == 1 else -1.0
        opt.step(params, [[sgn * g]])
        m_t = (1 - b1) * g * (-1.0) ** (t + 1) * (1 - (-b1) ** t) / (1 + b1)
        mhat = m_t / (1 - b1 ** t)
        expect = expect - lr * mhat / (np.abs(g) + eps)
        np.testing.assert_allclose(params[0][0], expect, rtol=1e-13, atol=1e-15)
