"""GPU checks at the benchmark's full sizes, in the launch configuration the
benchmark times (its own stream, so the time steps and sweeps replay HIP
graphs; launch shapes autotuned as the benchmark tunes them): the 1D job of
two N = 65536 problems and one 4096 x 4096 Sylvester step.  The oracle cannot
factor these sizes densely, so the 1D checks use its rows of M on sampled
outputs and the 2D check the full residual of the low-rank step against its
dense coefficient matrices."""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import fde1d as O
from oracle import fde2d as O2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N1 = 65536


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_05522_amd as H
    H.lib()
    return H


@pytest.fixture(scope="module")
def stream(H):
    return torch.cuda.Stream()


@pytest.fixture(scope="module")
def ctx(H, stream):
    return H.Context(stream)


def sample_rows(n, rng, count=40):
    edge = {0, 1, 2, 63, 64, 65, 66, n // 2, n - 67, n - 66, n - 65, n - 3, n - 2, n - 1}
    return sorted(edge | set(int(v) for v in rng.integers(0, n, count)))


def rows_of(p, rows):
    return O.fd_rows(p.alpha, p.n, p.nu, p.d_plus, p.d_minus, rows)


@pytest.fixture(scope="module")
def full_1d(H, ctx, stream):
    probs = [W.var_1d(1.2, n=N1), W.var_1d(1.8, n=N1)]
    with torch.cuda.stream(stream):
        ops = [H.operator_dict(p.n, p.alpha, p.dt, p.h, dev(p.d_plus), dev(p.d_minus)) for p in probs]
        At = H.HodlrMatrix(ctx, ops, H.default_opts(tol=1e-10, prec="fp32"))
        At.autotune()
        At.close()
        A = H.HodlrMatrix(ctx, ops, H.default_opts(tol=1e-10, prec="fp32", refine_max=3, rtol=1e-10))
    yield probs, A
    A.close()


def test_full_size_exact_operator_sampled_rows(full_1d, stream):
    """The exact product (near band in double-double + FFT far field) of the two
    65536-row operators equals, on sampled rows (the edges, the band's reach and
    random rows), the oracle's rows of M times x summed exactly (math.fsum of
    the rounded products), within 1e-12 of the row's sum of |M_ij x_j|."""
    probs, A = full_1d
    rng = np.random.default_rng(21)
    x = rng.standard_normal(2 * N1)
    with torch.cuda.stream(stream):
        y = torch.zeros(2 * N1, dtype=torch.float64, device="cuda")
        A.toeplitz_matvec(dev(x), y)
        stream.synchronize()
        y = y.cpu().numpy()
    for k, p in enumerate(probs):
        xs = x[k * N1:(k + 1) * N1]
        rows = sample_rows(N1, rng)
        R = rows_of(p, rows)
        for r, i in enumerate(rows):
            prod = R[r] * xs
            ref = math.fsum(prod.tolist())
            scale = math.fsum(np.abs(prod).tolist())
            assert abs(y[k * N1 + i] - ref) <= 1e-12 * scale, (k, i, y[k * N1 + i], ref, scale)


def test_full_size_refined_step_residual(full_1d, stream):
    """One implicit Euler step of both 65536-row problems with FP32 factors and
    three FP64 refinement sweeps (the benchmark's configuration, replayed from
    its HIP graph): on sampled rows the oracle's residual b - M u is below
    1e-10 of the row's sum of |M_ij u_j|."""
    probs, A = full_1d
    with torch.cuda.stream(stream):
        A.factor(allow=(0, 3))
        u = dev(np.concatenate([p.u0 for p in probs]))
        f = dev(np.concatenate([p.f for p in probs]))
        A.time_steps(u, f, probs[0].dt, 1, allow=(0, 2))
        stream.synchronize()
        u = u.cpu().numpy()
    rng = np.random.default_rng(22)
    for k, p in enumerate(probs):
        us = u[k * N1:(k + 1) * N1]
        b = p.u0 + p.dt * p.f
        rows = sample_rows(N1, rng)
        R = rows_of(p, rows)
        for r, i in enumerate(rows):
            prod = R[r] * us
            res = math.fsum([b[i]] + (-prod).tolist())
            scale = math.fsum(np.abs(prod).tolist()) + abs(b[i])
            assert abs(res) <= 1e-10 * scale, (k, i, res, scale)


@pytest.mark.parametrize("ek", [False, True], ids=["fadi", "ek"])
def test_full_size_sylvester_step_residual(H, ctx, stream, ek):
    """One step of the 4096 x 4096 workload (U^0 = 0, rank-4 source, FP32
    factors, tolerance 1e-10, sweeps replayed from their HIP graphs): the
    oracle's residual R = C - A X - X B^T of the low-rank result X = Z W^T,
    with the dense A and B of eq. (sylv-timestepping), gives a normwise
    backward error ||R||_F / ((a + b) ||X||_F + ||C||_F) below 1e-10, with
    a <= ||A||_2, b <= ||B||_2 the largest diagonal entries (so the test's
    figure bounds the true backward error from above), the step reports
    ||R||_F / ||C||_F as the test finds it, and the relative forward error
    against the oracle's step (stored by tests/golden/make_fd2d.py) is below
    1e-10.  The same with the extended Krylov solver (ek) in place of the
    fADI sweeps."""
    n = 4096
    p = W.fd_2d(n=n)
    with torch.cuda.stream(stream):
        opx = H.operator_dict(p.nx, p.alpha_x, p.dt, p.hx, dev(p.dxp), dev(p.dxm), 0.5)
        opy = H.operator_dict(p.ny, p.alpha_y, p.dt, p.hy, dev(p.dyp), dev(p.dym), 0.5)
        F = (dev(p.f.Z.T.copy()), dev(p.f.W.T.copy()))
        P = H.Fde2dPlan(ctx, opx, opy, H.default_opts(tol=1e-10, prec="fp32"), tol=1e-10, workspace=not ek)
        cur = (torch.zeros((0, n), dtype=torch.float64, device="cuda"),) * 2
        out = (torch.zeros((64, n), dtype=torch.float64, device="cuda"),
               torch.zeros((64, n), dtype=torch.float64, device="cuda"))
        r, info = P.step(cur, F, p.dt, out, ek=ek)
        stream.synchronize()
        Z = out[0][:r].cpu().numpy().T
        Wf = out[1][:r].cpu().numpy().T
        P.close()
    assert r > 0
    A, B = O2.sylvester_coefficients(p)
    C = p.dt * (p.f.Z @ p.f.W.T)
    X = Z @ Wf.T
    R = O2.residual(A, B, X, C)
    nr, nc, nx = np.linalg.norm(R), np.linalg.norm(C), np.linalg.norm(X)
    a, b = np.max(np.diag(A)), np.max(np.diag(B))
    eta = nr / ((a + b) * nx + nc)
    # forward error against the oracle's Bartels-Stewart step, stored as SVD
    # factors by tests/golden/make_fd2d.py
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fd2d_n4096.npz"))
    Xref = g["Z"] @ g["W"].T
    ferr = np.linalg.norm(X - Xref) / np.linalg.norm(Xref)
    print(f"4096^2 step: relative forward error against the oracle {ferr:.2e}")
    assert ferr <= 1e-10, ferr
    print(f"4096^2 step: rank {r}, ADI steps {info.refine_iters}, backward error {eta:.2e} "
          f"(reported {info.backward_error:.2e}), ||R||/||C|| {nr / nc:.2e} (reported {info.rel_residual:.2e}), "
          f"last correction {info.rel_correction:.2e}")
    assert eta <= 1e-10, (eta, nr / nc, r, info.refine_iters, info.rel_correction)
    assert abs(info.rel_residual - nr / nc) <= 0.05 * nr / nc + 1e-14, (info.rel_residual, nr / nc)


@pytest.mark.parametrize("ek", [False, True], ids=["fadi", "ek"])
def test_full_size_fe_sylvester_step(H, ctx, stream, ek):
    """One step of the paper's finite-element workload at 4096 x 4096 (P1
    elements, alpha = (1.3, 1.7), dt = 0.1, U^0 = F = indicator of
    [3/8, 5/8]^2) with the benchmark's options (FP32 factors, tolerance
    1e-10), against the oracle's step stored by tests/golden/make_fe2d.py
    (Bartels-Stewart on the mass-reduced matrices plus one refinement step):
    relative forward error below 1e-10, and the normwise backward error of the
    generalized equation, formed from the oracle's dense A and B and the
    tridiagonal mass matrices (||A||, ||B||, ||E|| replaced by their largest
    diagonal entries), below 1e-10.  The same with the extended Krylov
    solver (ek) on the pencils."""
    from oracle import fe as OF
    n = 4096
    p = W.fe_2d(n=n)
    with torch.cuda.stream(stream):
        opx = H.operator_dict(p.nx, p.alpha_x, p.dt, p.hx, dev(p.dxp), dev(p.dxm), 0.5, discretization=H.FDE_FE)
        opy = H.operator_dict(p.ny, p.alpha_y, p.dt, p.hy, dev(p.dyp), dev(p.dym), 0.5, discretization=H.FDE_FE)
        P = H.Fde2dPlan(ctx, opx, opy, H.default_opts(tol=1e-10, prec="fp32"), tol=1e-10, workspace=not ek)
        cur = (dev(p.u0.Z.T.copy()), dev(p.u0.W.T.copy()))
        F = (dev(p.f.Z.T.copy()), dev(p.f.W.T.copy()))
        out = (torch.zeros((64, n), dtype=torch.float64, device="cuda"),
               torch.zeros((64, n), dtype=torch.float64, device="cuda"))
        r, info = P.step(cur, F, p.dt, out, ek=ek)
        stream.synchronize()
        Z = out[0][:r].cpu().numpy().T
        Wf = out[1][:r].cpu().numpy().T
        P.close()
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fe2d_n4096.npz"))
    Xref = g["Z"] @ g["W"].T
    X = Z @ Wf.T
    ferr = np.linalg.norm(X - Xref) / np.linalg.norm(Xref)
    A, B, _, _ = OF.fe_sylvester_coefficients(p)
    C = OF.mass_apply(OF.mass_apply(p.u0.dense() + p.dt * p.f.dense()).T).T
    R = C - (A @ Z) @ OF.mass_apply(Wf).T - OF.mass_apply(Z) @ (B @ Wf).T     # C - A X E_y - E_x X B^T
    a, b = np.max(np.diag(A)), np.max(np.diag(B))
    eta = np.linalg.norm(R) / ((a + b) * (2 / 3) * np.linalg.norm(X) + np.linalg.norm(C))
    print(f"fe 4096^2 step: rank {r}, ADI steps {info.refine_iters}, forward error {ferr:.2e}, "
          f"backward error {eta:.2e} (reported {info.backward_error:.2e}), last correction {info.rel_correction:.2e}")
    assert ferr <= 1e-10, ferr
    assert eta <= 1e-10, eta


def test_full_size_batched_step_sampled_rows(H, ctx, stream):
    """The batched workload (256 ragged problems, N from 2048 to 32768, small
    and four-step transform lengths in one batch) in the benchmark's
    configuration: for a spread of problems, sampled rows of the exact product
    match the oracle's rows of M (within 1e-12 of the row's sum of |M_ij x_j|)
    and, after one refined FP32 step, the oracle's residual rows are below
    1e-10 of the row's sum of |M_ij u_j|."""
    probs = W.batched_1d()
    ns = np.array([p.n for p in probs])
    off = np.concatenate([[0], np.cumsum(ns)])
    total = int(off[-1])
    pick = sorted({int(np.argmin(ns)), int(np.argmax(ns)), 0, 77, 128, 255})
    rng = np.random.default_rng(23)
    x = rng.standard_normal(total)
    with torch.cuda.stream(stream):
        ops = [H.operator_dict(p.n, p.alpha, p.dt, p.h, dev(p.d_plus), dev(p.d_minus)) for p in probs]
        At = H.HodlrMatrix(ctx, ops, H.default_opts(tol=1e-10, prec="fp32"))
        At.autotune()
        At.close()
        A = H.HodlrMatrix(ctx, ops, H.default_opts(tol=1e-10, prec="fp32", refine_max=3, rtol=1e-10))
        y = torch.zeros(total, dtype=torch.float64, device="cuda")
        A.toeplitz_matvec(dev(x), y)
        A.factor(allow=(0, 3))
        u = dev(np.concatenate([p.u0 for p in probs]))
        f = dev(np.concatenate([p.f for p in probs]))
        A.time_steps(u, f, probs[0].dt, 1, allow=(0, 2))
        stream.synchronize()
        y = y.cpu().numpy()
        u = u.cpu().numpy()
        A.close()
    for k in pick:
        p, lo = probs[k], int(off[k])
        rows = sample_rows(p.n, rng, count=16)
        R = rows_of(p, rows)
        xs, us = x[lo:lo + p.n], u[lo:lo + p.n]
        b = p.u0 + p.dt * p.f
        for r, i in enumerate(rows):
            prod = R[r] * xs
            assert abs(y[lo + i] - math.fsum(prod.tolist())) <= 1e-12 * math.fsum(np.abs(prod).tolist()), (k, i)
            prod = R[r] * us
            res = math.fsum([b[i]] + (-prod).tolist())
            assert abs(res) <= 1e-10 * (math.fsum(np.abs(prod).tolist()) + abs(b[i])), (k, i, res)


def test_full_size_time_dependent_steps_sampled_rows(H, ctx, stream):
    """The time-dependent workload at full size, as the benchmark runs it:
    the 256 ragged problems rebuilt in place for new coefficients, factored
    and solved with three FP64 refinement sweeps, two steps.  After the second
    step the oracle's residual rows of M(t_2) (built from the step's own
    coefficient samples) are below 1e-10 of the row's sum of |M_ij u_j| on
    sampled rows of a spread of problems."""
    probs = W.batched_1d()
    ns = np.array([p.n for p in probs])
    off = np.concatenate([[0], np.cumsum(ns)])
    dt = probs[0].dt
    coefs = [[W.timedep_coefficients(p, m * p.dt) for p in probs] for m in range(3)]
    with torch.cuda.stream(stream):
        dco = [[(dev(a), dev(b)) for a, b in c] for c in coefs]
        ops = [[H.operator_dict(p.n, p.alpha, p.dt, p.h, a, b) for p, (a, b) in zip(probs, c)] for c in dco]
        A = H.HodlrMatrix(ctx, ops[0], H.default_opts(tol=1e-10, prec="fp32", refine_max=3, rtol=1e-10))
        u = dev(np.concatenate([p.u0 for p in probs]))
        f = dev(np.concatenate([p.f for p in probs]))
        rhs = torch.empty_like(u)
        prev = None
        for m in (1, 2):
            A.update_coefficients(ops[m])
            A.factor(allow=(0, 3))
            torch.add(u, f, alpha=dt, out=rhs)
            A.solve(rhs, allow=(0, 2))
            stream.synchronize()
            prev = u.cpu().numpy()
            u.copy_(rhs)
        stream.synchronize()
        u = u.cpu().numpy()
        A.close()
    rng = np.random.default_rng(24)
    for k in sorted({int(np.argmin(ns)), int(np.argmax(ns)), 3, 200}):
        p, lo = probs[k], int(off[k])
        dp, dm = coefs[2][k]
        rows = sample_rows(p.n, rng, count=16)
        R = O.fd_rows(p.alpha, p.n, p.nu, dp, dm, rows)
        b = prev[lo:lo + p.n] + dt * p.f
        us = u[lo:lo + p.n]
        for r, i in enumerate(rows):
            prod = R[r] * us
            res = math.fsum([b[i]] + (-prod).tolist())
            assert abs(res) <= 1e-10 * (math.fsum(np.abs(prod).tolist()) + abs(b[i])), (k, i, res)
