"""GPU parity of the finite-element path (Sec. 2.2.2, Sec. 3.4.3, eq.
(sylv-timestepping-fe)) against the finite-element oracle, through the C ABI:
the exact operator (with the mass matrix), the HODLR compression of the
P1 stiffness (shifted Hankel plus the exact first block row), factor and
solve in FP64 and mixed precision, the time loop, and the 2D generalized
Sylvester step by generalized factored ADI on the paper's finite-element
workload."""
import numpy as np
import pytest

import workloads as W
from oracle import fde1d as O
from oracle import fe as OF

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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
def ctx(H):
    return H.Context()


def fe_problem(n, alpha, dt=1 / 64, seed=0, variable=False):
    x, h = W.grid(n)
    rng = np.random.default_rng(seed)
    if variable:     # row-scaled reading of variable coefficients
        dp = 1 + x * x + 0.1 * rng.random(n)
        dm = 1 + (1 - x) ** 2
    else:
        dp = dm = np.full(n, 1.3)
    return W.Problem1D(n, alpha, dt, 4, h, x, dp, dm, W.bump(x), W.gaussian_source(x, rng))


def build(H, ctx, probs, shift=1.0, **kw):
    ops = [H.operator_dict(p.n, p.alpha, p.dt, p.h, dev(p.d_plus), dev(p.d_minus), shift,
                           discretization=H.FDE_FE) for p in probs]
    return H.HodlrMatrix(ctx, ops, H.default_opts(**kw))


@pytest.mark.parametrize("alpha", [1.1, 1.3, 1.7, 1.9, 2.0])
def test_weights_match_oracle(H, ctx, alpha):
    """The P1 stiffness generator the library computes (double-double
    arithmetic, rounded once) equals the oracle's multi-precision weights:
    at most 1 ulp apart, and in all but a few near-ties bit for bit.  The
    finite-difference weights of the same batch (the product recursion, as a
    blocked scan on the device and sequentially in the oracle) agree to the
    rounding the recursion accumulates."""
    n = 70000
    x, h = W.grid(n)
    one = dev(np.ones(n))
    ops = [H.operator_dict(n, alpha, 0.1, h, one, one, 1.0, discretization=H.FDE_FE),
           H.operator_dict(n, alpha, 0.1, h, one, one, 1.0)]
    A = H.HodlrMatrix(ctx, ops, H.default_opts(tol=1e-10))
    w = A.weights(0, n + 3)
    ref = OF.fe_weights(alpha, n + 3)
    zero = ref == 0.0
    assert np.all(np.abs(w[zero]) <= 1e-28)          # alpha = 2: exact zeros beyond w_2
    nz = ~zero
    ulps = np.abs(w[nz] - ref[nz]) / np.spacing(np.abs(ref[nz]))
    print(f"alpha={alpha}: {int(np.count_nonzero(ulps))} of {int(nz.sum())} weights 1 ulp from the oracle")
    assert ulps.max() <= 1.0 and np.count_nonzero(ulps) <= 1e-3 * nz.sum()
    g, gref = A.weights(1, n + 3), O.gl_weights(alpha, n + 2)
    gz = gref == 0.0
    assert np.all(g[gz] == 0.0)
    rel = np.max(np.abs(g[~gz] - gref[~gz]) / np.abs(gref[~gz]))
    print(f"alpha={alpha}: finite-difference weights within {rel:.1e} of the oracle's recursion")
    assert rel <= 1e-13
    A.close()


@pytest.mark.parametrize("n", [1, 2, 5, 300, 4096, 5000])
@pytest.mark.parametrize("alpha", [1.3, 1.7])
def test_exact_operator_matches_double_double(H, ctx, n, alpha):
    """The exact product of s E + nu (D+ T + D- T^T) (near band and mass in
    double-double, far field by FFT) equals the oracle's double-double
    residual to a few ulps of |M||x|; the weights the device computes
    (direct sum near the diagonal, series away from it) enter every entry."""
    p = fe_problem(n, alpha, variable=True)
    A = build(H, ctx, [p], shift=0.75)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(n)
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    A.toeplitz_matvec(dev(x), y)
    ref = -OF.residual_dd(alpha, p.nu, 0.75, p.d_plus, p.d_minus, x, np.zeros(n))
    w = OF.fe_weights(alpha, n + 2)
    aw = np.abs(w[:n + 1])
    absM_x = 0.75 * OF.mass_apply(np.abs(x)) + p.nu * (
        p.d_plus * np.convolve(np.abs(x), aw, "full")[1:n + 1]
        + p.d_minus * np.convolve(np.abs(x)[::-1], aw, "full")[1:n + 1][::-1])
    rel = np.max(np.abs(y.cpu().numpy() - ref) / absM_x)
    assert rel < 1e-13, rel


@pytest.mark.parametrize("n", [40, 65])
@pytest.mark.parametrize("kind", ["fd", "fe"])
def test_near_band_product_is_double_double(H, ctx, n, kind):
    """For n <= 65 the whole product lies in the near band, which is summed
    in double-double: every entry of M x is within an ulp or two of the
    oracle's double-double value (not merely of |M| |x|), for both
    discretizations."""
    rng = np.random.default_rng(n)
    p = fe_problem(n, 1.45, variable=True, seed=n)
    x = rng.standard_normal(n)
    if kind == "fe":
        A = build(H, ctx, [p], shift=0.75)
        ref = -OF.residual_dd(1.45, p.nu, 0.75, p.d_plus, p.d_minus, x, np.zeros(n))
    else:
        ops = [H.operator_dict(n, 1.45, p.dt, p.h, dev(p.d_plus), dev(p.d_minus), 0.75)]
        A = H.HodlrMatrix(ctx, ops, H.default_opts())
        ref = -O.residual_dd(1.45, p.nu, 0.75, p.d_plus, p.d_minus, x, np.zeros(n))
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    A.toeplitz_matvec(dev(x), y)
    ulps = np.abs(y.cpu().numpy() - ref) / np.spacing(np.abs(ref))
    assert ulps.max() <= 2, ulps.max()


@pytest.mark.parametrize("n", [17, 64, 65, 777, 2049])
@pytest.mark.parametrize("alpha", [1.3, 1.7])
def test_compressed_operator_matches_dense(H, ctx, n, alpha):
    """The HODLR representation (Hankel [w_{p+q+3}] factored, first block rows
    exact, mass in the leaves and corners): ||M_H x - M x|| <= c eps ||M||_2 ||x||."""
    p = fe_problem(n, alpha, variable=True)
    eps = 1e-10
    A = build(H, ctx, [p], tol=eps)
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, 3))
    y = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    A.matvec(dev(X.T).contiguous(), y, nrhs=3, ld=n)
    M = OF.fe_matrix(alpha, n, p.nu, p.d_plus, p.d_minus, 1.0)
    err = np.linalg.norm(y.cpu().numpy().T - M @ X, 2)
    bound = 20 * eps * np.linalg.norm(M, 2) * np.linalg.norm(X, 2)
    assert err <= bound, (err, bound)


@pytest.mark.parametrize("alpha", [1.3, 1.7])
def test_operator_rank_near_dense_eps_rank(H, ctx, alpha):
    """Off-diagonal rank of the compressed finite-element operator: at most 2
    above the dense eps-rank of the top-level blocks at the same tau."""
    n, eps = 4096, 1e-10
    p = fe_problem(n, alpha, dt=0.1)
    A = build(H, ctx, [p], tol=eps)
    rA = A.info().max_rank_A
    M = OF.fe_matrix(alpha, n, p.nu, p.d_plus, p.d_minus, 1.0)
    tau = eps * np.max(np.abs(np.diag(M)))
    n1 = n // 2
    dense = max(O.eps_rank(M[n1:, :n1], tau), O.eps_rank(M[:n1, n1:], tau))
    print(f"alpha={alpha}: operator rank {rA}, dense eps-rank {dense}")
    assert rA <= dense + 2, (rA, dense)


@pytest.mark.parametrize("n,alpha,prec", [(1000, 1.3, "fp64"), (3001, 1.7, "fp64"),
                                          (3001, 1.3, "fp32"), (3001, 1.7, "bf16")])
def test_factor_solve(H, ctx, n, alpha, prec):
    """HODLR LU + solve of the finite-element matrix vs the oracle's refined
    dense solve: FP64 factors (two refinement sweeps) <= 1e-8; reduced-precision
    factors with FP64 refinement (GMRES-IR for BF16) <= 1e-10 without fallback."""
    p = fe_problem(n, alpha, dt=1 / 16)
    kw = dict(tol=1e-10, refine_max=2 if prec == "fp64" else 8, rtol=1e-12)
    if prec == "bf16":
        kw["gmres_m"] = 8
    A = build(H, ctx, [p], prec=prec, **kw)
    A.factor()
    b = np.sin(5 * p.x) + p.f
    x = dev(b)
    info = A.solve(x, allow=(0, 2))
    ref = OF.FeSolver(alpha, n, p.nu, p.d_plus, p.d_minus).solve(b)
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"n={n} alpha={alpha} {prec}: rel.err {err:.2e} sweeps {info.refine_iters} fallback {info.used_fallback}")
    assert err <= (1e-8 if prec == "fp64" else 1e-10), err
    if prec != "fp64":
        assert info.used_fallback == 0


def test_time_steps_fe_workload(H, ctx):
    """The 1D finite-element workload (N = 4096, alpha = 1.3, 16 steps of
    (E + nu (...)) u^m = E (u^(m-1) + dt f)) in the graph time loop with FP32
    factors and three refinement sweeps a step, against the oracle's steps:
    rel. error <= 1e-10, no fallback."""
    p = W.fe_1d()
    A = build(H, ctx, [p], prec="fp32", tol=1e-10, refine_max=3, rtol=1e-10)
    A.factor()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        A.ctx = H.Context(stream)
        u = dev(p.u0)
        info = A.time_steps(u, dev(p.f), p.dt, p.steps)
        stream.synchronize()
    ref = OF.euler_fe_1d(p)
    err = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"fe_1d: rel.err {err:.2e}, worst correction {info.rel_correction:.2e}, fallback {info.used_fallback}")
    assert err <= 1e-10 and info.used_fallback == 0, (err, info.used_fallback)


def test_batched_fd_and_fe_problems(H, ctx):
    """One batch mixing finite-difference and finite-element operators gives
    each problem's own solution (the time-step right-hand side applies the
    mass matrix to the finite-element problems only)."""
    pf = fe_problem(900, 1.4, seed=5)
    pd = fe_problem(1300, 1.6, seed=6)
    ops = [H.operator_dict(pd.n, pd.alpha, pd.dt, pd.h, dev(pd.d_plus), dev(pd.d_minus), 1.0),
           H.operator_dict(pf.n, pf.alpha, pf.dt, pf.h, dev(pf.d_plus), dev(pf.d_minus), 1.0,
                           discretization=H.FDE_FE)]
    A = H.HodlrMatrix(ctx, ops, H.default_opts(tol=1e-12, refine_max=2, rtol=1e-13))
    A.factor()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        A.ctx = H.Context(stream)
        u = dev(np.concatenate([pd.u0, pf.u0]))
        f = dev(np.concatenate([pd.f, pf.f]))
        A.time_steps(u, f, 1 / 64, 3, allow=(0, 2))
        stream.synchronize()
    got = u.cpu().numpy()
    ref_d = O.euler_1d(pd, steps=3)
    ref_f = OF.euler_fe_1d(pf, steps=3)
    assert np.linalg.norm(got[:pd.n] - ref_d) <= 1e-10 * np.linalg.norm(ref_d)
    assert np.linalg.norm(got[pd.n:] - ref_f) <= 1e-10 * np.linalg.norm(ref_f)


def lr_dev(Z, W_):
    return dev(Z.T.copy()), dev(W_.T.copy())


def fe_plan(H, ctx, p, prec="fp64", tol=1e-10, hodlr_tol=1e-12, leaf=32, workspace=True):
    opx = H.operator_dict(p.nx, p.alpha_x, p.dt, p.hx, dev(p.dxp), dev(p.dxm), 0.5, discretization=H.FDE_FE)
    opy = H.operator_dict(p.ny, p.alpha_y, p.dt, p.hy, dev(p.dyp), dev(p.dym), 0.5, discretization=H.FDE_FE)
    return H.Fde2dPlan(ctx, opx, opy, H.default_opts(tol=hodlr_tol, prec=prec, leaf=leaf), tol=tol,
                       workspace=workspace)


@pytest.mark.parametrize("n,prec", [(150, "fp64"), (512, "fp64"), (1024, "fp32")])
def test_2d_fe_steps_match_oracle(H, ctx, n, prec):
    """Steps of the paper's finite-element workload (alpha = (1.3, 1.7),
    dt = 0.1, f = u0 = indicator of [3/8, 5/8]^2) by generalized factored ADI
    (shifted solves with A + q E_x, residual updates through E, no inverse
    mass matrix) against the oracle's route (mass matrices inverted, then
    Bartels-Stewart), step tolerance 1e-10.  The normwise backward error of
    the generalized equation, formed densely from the oracle's matrices, is
    below 1e-10; the forward error is below 1e-8 with FP64 factors (one sweep
    reaching the backward-error target; at dt = 0.1 the smooth modes keep
    errors the backward error does not weigh) and below 1e-10 with FP32
    factors, whose corrections run until the last one is below 1e-10."""
    tol = 1e-10
    p = W.fe_2d(n=n)
    P = fe_plan(H, ctx, p, prec=prec, tol=tol, hodlr_tol=1e-10 if prec != "fp64" else 1e-12)
    st = OF.FeSylvesterStepper(p)
    na, nb = np.linalg.norm(st.A, 2), np.linalg.norm(st.B, 2)
    ne_x, ne_y = np.linalg.norm(st.Ex, 2), np.linalg.norm(st.Ey, 2)
    U = p.u0.dense()
    cur = lr_dev(p.u0.Z, p.u0.W)
    for k in range(3):
        out = (torch.zeros((64, n), dtype=torch.float64, device="cuda"),
               torch.zeros((64, n), dtype=torch.float64, device="cuda"))
        r, info = P.step(cur, lr_dev(p.f.Z, p.f.W), p.dt, out)
        X = out[0][:r].cpu().numpy().T @ out[1][:r].cpu().numpy()
        C = st.rhs(U, p.f.dense())
        U = st.step(U, p.f.dense())
        err = np.linalg.norm(X - U) / np.linalg.norm(U)
        R = OF.generalized_residual(st.A, st.B, st.Ex, st.Ey, X, C)
        eta = np.linalg.norm(R) / ((na * ne_y + ne_x * nb) * np.linalg.norm(X) + np.linalg.norm(C))
        res = np.linalg.norm(R) / np.linalg.norm(C)
        print(f"fe_2d n={n} {prec} step {k + 1}: rank {r} adi {info.refine_iters} rel.err {err:.2e} "
              f"backward error {eta:.2e} (reported {info.backward_error:.2e}) ||R||/||C|| {res:.2e} "
              f"(reported {info.rel_residual:.2e})")
        assert err <= (1e-8 if prec == "fp64" else 1e-10) and eta <= tol, (err, eta)
        assert abs(info.rel_residual - res) <= 0.05 * res + 1e-14, (info.rel_residual, res)
        cur = (out[0][:r].contiguous(), out[1][:r].contiguous())
    P.close()


@pytest.mark.parametrize("n,prec", [(150, "fp64"), (512, "fp32")])
def test_2d_fe_extended_krylov(H, ctx, n, prec):
    """The finite-element steps by extended Krylov (Sec. 4.3) on the pencils:
    bases of EK(E_x^-1 A, E_x^-1 G) and EK(E_y^-1 B, E_y^-1 H) (exact
    products followed by tridiagonal mass solves; inverses as refined HODLR
    solves of A after a mass product), three steps against the oracle's
    route, forward error and the dense normwise backward error of the
    generalized equation below 1e-10."""
    tol = 1e-10
    p = W.fe_2d(n=n)
    P = fe_plan(H, ctx, p, prec=prec, tol=tol, hodlr_tol=1e-10 if prec != "fp64" else 1e-12, workspace=False)
    st = OF.FeSylvesterStepper(p)
    na, nb = np.linalg.norm(st.A, 2), np.linalg.norm(st.B, 2)
    ne_x, ne_y = np.linalg.norm(st.Ex, 2), np.linalg.norm(st.Ey, 2)
    U = p.u0.dense()
    cur = lr_dev(p.u0.Z, p.u0.W)
    for k in range(3):
        out = (torch.zeros((64, n), dtype=torch.float64, device="cuda"),
               torch.zeros((64, n), dtype=torch.float64, device="cuda"))
        r, info = P.step(cur, lr_dev(p.f.Z, p.f.W), p.dt, out, ek=True)
        X = out[0][:r].cpu().numpy().T @ out[1][:r].cpu().numpy()
        C = st.rhs(U, p.f.dense())
        U = st.step(U, p.f.dense())
        err = np.linalg.norm(X - U) / np.linalg.norm(U)
        R = OF.generalized_residual(st.A, st.B, st.Ex, st.Ey, X, C)
        eta = np.linalg.norm(R) / ((na * ne_y + ne_x * nb) * np.linalg.norm(X) + np.linalg.norm(C))
        print(f"fe_2d ek n={n} {prec} step {k + 1}: rank {r} iterations {info.refine_iters} rel.err {err:.2e} "
              f"backward error {eta:.2e} (reported {info.backward_error:.2e})")
        assert err <= tol and eta <= tol, (err, eta)
        cur = (out[0][:r].contiguous(), out[1][:r].contiguous())
    P.close()


def test_update_coefficients_fe(H, ctx):
    """hodlr_update_coefficients on a finite-element operator: new d+/d-
    samples rebuild the compression and leaves (the generator and the mass
    terms stay), and the refactored solve matches the oracle's matrix with
    the new coefficients."""
    p = fe_problem(1500, 1.5, seed=9)
    A = build(H, ctx, [p], tol=1e-12, refine_max=2, rtol=1e-13)
    x, h = W.grid(p.n)
    dp2, dm2 = 1.0 + 0.5 * x, 2.0 - x
    A.update_coefficients([H.operator_dict(p.n, p.alpha, p.dt, p.h, dev(dp2), dev(dm2), 1.0,
                                           discretization=H.FDE_FE)])
    A.factor()
    b = np.cos(4 * p.x)
    xs = dev(b)
    A.solve(xs, allow=(0, 2))
    ref = OF.FeSolver(p.alpha, p.n, p.nu, dp2, dm2).solve(b)
    assert np.linalg.norm(xs.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    with pytest.raises(H.HodlrError):      # the discretization cannot change in place
        A.update_coefficients([H.operator_dict(p.n, p.alpha, p.dt, p.h, dev(dp2), dev(dm2), 1.0)])


def test_2d_fe_variable_coefficients(H, ctx):
    """The generalized step with variable (row-scaled) coefficients, eq.
    (coeff_es) samples on both axes: the pencils' intervals assume a
    coercive stiffness form, which row scaling does not guarantee; the step
    still meets its backward-error tolerance and matches the oracle."""
    n = 150
    p = W.fe_2d(n=n)
    import math
    g12 = math.gamma(1.2)
    p.dxp, p.dxm = g12 * (1 + p.x) ** p.alpha_x, g12 * (2 - p.x) ** p.alpha_x
    p.dyp, p.dym = g12 * (1 + p.y) ** p.alpha_y, g12 * (2 - p.y) ** p.alpha_y
    P = fe_plan(H, ctx, p, tol=1e-10)
    st = OF.FeSylvesterStepper(p)
    out = (torch.zeros((64, n), dtype=torch.float64, device="cuda"),
           torch.zeros((64, n), dtype=torch.float64, device="cuda"))
    r, info = P.step(lr_dev(p.u0.Z, p.u0.W), lr_dev(p.f.Z, p.f.W), p.dt, out)
    X = out[0][:r].cpu().numpy().T @ out[1][:r].cpu().numpy()
    U = st.step(p.u0.dense(), p.f.dense())
    err = np.linalg.norm(X - U) / np.linalg.norm(U)
    print(f"fe_2d variable coefficients n={n}: adi {info.refine_iters} rel.err {err:.2e} "
          f"backward error {info.backward_error:.2e}")
    assert info.backward_error <= 1e-10 and err <= 1e-8, (err, info.backward_error)
    P.close()


@pytest.mark.parametrize("ek", [False, True], ids=["fadi", "ek"])
@pytest.mark.parametrize("alphas", [(1.1, 1.9), (1.9, 1.1)])
def test_2d_fe_both_solvers_across_orders(H, ctx, alphas, ek):
    """The finite-element step with both solvers at the ends of the orders'
    range (n = 150, FP32 factors, tolerance 1e-10): two steps against the
    oracle's route, forward error and the dense generalized backward error
    below 1e-10."""
    tol = 1e-10
    p = W.fe_2d(n=150, alpha_x=alphas[0], alpha_y=alphas[1])
    P = fe_plan(H, ctx, p, prec="fp32", tol=tol, hodlr_tol=1e-10)
    st = OF.FeSylvesterStepper(p)
    na, nb = np.linalg.norm(st.A, 2), np.linalg.norm(st.B, 2)
    ne_x, ne_y = np.linalg.norm(st.Ex, 2), np.linalg.norm(st.Ey, 2)
    U = p.u0.dense()
    cur = lr_dev(p.u0.Z, p.u0.W)
    for k in range(2):
        out = (torch.zeros((64, p.nx), dtype=torch.float64, device="cuda"),
               torch.zeros((64, p.ny), dtype=torch.float64, device="cuda"))
        r, info = P.step(cur, lr_dev(p.f.Z, p.f.W), p.dt, out, ek=ek)
        X = out[0][:r].cpu().numpy().T @ out[1][:r].cpu().numpy()
        C = st.rhs(U, p.f.dense())
        U = st.step(U, p.f.dense())
        err = np.linalg.norm(X - U) / np.linalg.norm(U)
        R = OF.generalized_residual(st.A, st.B, st.Ex, st.Ey, X, C)
        eta = np.linalg.norm(R) / ((na * ne_y + ne_x * nb) * np.linalg.norm(X) + np.linalg.norm(C))
        print(f"fe alphas {alphas} {'ek' if ek else 'fadi'} step {k + 1}: rel.err {err:.2e} backward error {eta:.2e}")
        assert err <= tol and eta <= tol, (err, eta)
        cur = (out[0][:r].contiguous(), out[1][:r].contiguous())
    P.close()


@pytest.mark.parametrize("ek", [False, True], ids=["fadi", "ek"])
@pytest.mark.parametrize("n", [1, 5, 33])
def test_2d_fe_tiny_grids(H, ctx, n, ek):
    """The finite-element step on grids of one point, of fewer points than a
    leaf, and of one point more than the plans' leaf of 32 (two leaves of
    16 and 17), with both solvers (FP32 factors, tolerance 1e-10): two steps
    against the oracle's route, forward error and the dense generalized
    backward error below 1e-10."""
    tol = 1e-10
    p = W.fe_2d(n=n)
    P = fe_plan(H, ctx, p, prec="fp32", tol=tol, hodlr_tol=1e-10)
    st = OF.FeSylvesterStepper(p)
    na, nb = np.linalg.norm(st.A, 2), np.linalg.norm(st.B, 2)
    ne_x, ne_y = np.linalg.norm(st.Ex, 2), np.linalg.norm(st.Ey, 2)
    U = p.u0.dense()
    cur = lr_dev(p.u0.Z, p.u0.W)
    for k in range(2):
        out = (torch.zeros((64, p.nx), dtype=torch.float64, device="cuda"),
               torch.zeros((64, p.ny), dtype=torch.float64, device="cuda"))
        r, info = P.step(cur, lr_dev(p.f.Z, p.f.W), p.dt, out, ek=ek)
        X = out[0][:r].cpu().numpy().T @ out[1][:r].cpu().numpy()
        C = st.rhs(U, p.f.dense())
        U = st.step(U, p.f.dense())
        err = np.linalg.norm(X - U) / np.linalg.norm(U)
        R = OF.generalized_residual(st.A, st.B, st.Ex, st.Ey, X, C)
        eta = np.linalg.norm(R) / ((na * ne_y + ne_x * nb) * np.linalg.norm(X) + np.linalg.norm(C))
        print(f"fe n={n} {'ek' if ek else 'fadi'} step {k + 1}: rel.err {err:.2e} backward error {eta:.2e} rank {r}")
        assert err <= tol and eta <= tol, (err, eta)
        cur = (out[0][:r].contiguous(), out[1][:r].contiguous())
    P.close()
