"""GPU parity of the 1D HODLR path (build, exact operator, factor, solve, time steps)
against the CPU oracle, through the C ABI."""
import numpy as np
import pytest

import workloads as W
from oracle import fde1d as O

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


def var_problem(n, alpha, dt=1 / 64, seed=0):
    x, h = W.grid(n)
    rng = np.random.default_rng(seed)
    dp = 1 + x * x + 0.1 * rng.random(n)
    dm = 1 + (1 - x) ** 2
    return W.Problem1D(n, alpha, dt, 4, h, x, dp, dm, W.bump(x), np.zeros(n))


def build(H, ctx, probs, **kw):
    ops = [H.operator_dict(p.n, p.alpha, p.dt, p.h, dev(p.d_plus), dev(p.d_minus), kw.pop("shift", 1.0))
           for p in probs]
    return H.HodlrMatrix(ctx, ops, H.default_opts(**kw))


SIZES = [1, 17, 64, 65, 200, 777, 1024, 2049]


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("alpha", [1.2, 1.8])
def test_compressed_operator_matches_dense(H, ctx, n, alpha):
    """HODLR representation of M (Sec. 3.4.2): ||M_H x - M x|| <= c eps ||M||_2 ||x||."""
    p = var_problem(n, alpha)
    eps = 1e-10
    A = build(H, ctx, [p], tol=eps)
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, 3))
    y = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    A.matvec(dev(X.T).contiguous(), y, nrhs=3, ld=n)
    M = O.fd_matrix(alpha, n, p.nu, p.d_plus, p.d_minus)
    ref = M @ X
    err = np.linalg.norm(y.cpu().numpy().T - ref, 2)
    bound = 20 * eps * np.linalg.norm(M, 2) * np.linalg.norm(X, 2)
    assert err <= bound, (err, bound)


@pytest.mark.parametrize("n", [2049, 4096])
@pytest.mark.parametrize("alpha", [1.2, 1.5, 1.8])
def test_operator_rank_near_dense_eps_rank(H, ctx, n, alpha):
    """The off-diagonal rank of the compressed operator (Sec. 3.4.1: blocks
    truncated at tau = eps ||M||_2, ||M||_2 taken from its lower bound
    max_i M_ii = 1 + nu alpha max(d+ + d-)) is at most 2 above the dense
    eps-rank of the top-level blocks at the same tau (dense SVD of the
    oracle's M), and the compressed operator keeps its accuracy."""
    p = W.var_1d(alpha, n=n)
    eps = 1e-10
    A = build(H, ctx, [p], tol=eps)
    rA = A.info().max_rank_A
    M = O.fd_matrix(alpha, n, p.nu, p.d_plus, p.d_minus)
    tau = eps * (1 + p.nu * alpha * np.max(p.d_plus + p.d_minus))
    n1 = n // 2
    dense = max(O.eps_rank(M[n1:, :n1], tau), O.eps_rank(M[:n1, n1:], tau))
    assert rA <= dense + 2, (rA, dense)
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, 2))
    y = torch.zeros((2, n), dtype=torch.float64, device="cuda")
    A.matvec(dev(X.T).contiguous(), y, nrhs=2, ld=n)
    err = np.linalg.norm(y.cpu().numpy().T - M @ X, 2)
    assert err <= 20 * eps * np.linalg.norm(M, 2) * np.linalg.norm(X, 2)
    print(f"n={n} alpha={alpha}: operator rank {rA}, dense eps-rank {dense}")


@pytest.mark.parametrize("n", [1, 5, 300, 4096, 5000, 20000])
@pytest.mark.parametrize("alpha", [1.1, 1.5, 1.9])
def test_exact_operator_matches_double_double(H, ctx, n, alpha):
    """Near-field double-double + far-field FFT product equals the oracle's
    double-double residual to a few ulps of |M||x| (both the single-pass and the
    four-step FFT lengths)."""
    p = var_problem(n, alpha)
    A = build(H, ctx, [p])
    rng = np.random.default_rng(1)
    x = rng.standard_normal(n)
    y = torch.zeros(n, dtype=torch.float64, device="cuda")
    A.toeplitz_matvec(dev(x), y)
    ref = -O.residual_dd(alpha, p.nu, 1.0, p.d_plus, p.d_minus, x, np.zeros(n))
    g = O.gl_weights(alpha, n + 1)
    # |M| |x| without forming M: |T| = T with signs flipped except g_1
    absM_x = np.abs(x) + p.nu * (p.d_plus * np.abs(np.convolve(np.abs(x), np.abs(g[:n + 1]), "full")[1:n + 1])
                                 + p.d_minus * np.abs(np.convolve(np.abs(x)[::-1], np.abs(g[:n + 1]), "full")[1:n + 1][::-1]))
    rel = np.max(np.abs(y.cpu().numpy() - ref) / absM_x)
    assert rel < 1e-13, rel


def test_exact_operator_many_transforms_in_one_launch(H, ctx):
    """48 four-step transforms (lengths 2^15 and 2^16) in one batch: the passes
    launch far more work-groups than are resident at once, so an output that
    lands in another work-group's input would show.  Repeated products agree
    bit for bit, every problem's product equals that problem's product alone,
    and the two shortest match the oracle's double-double residual."""
    rng = np.random.default_rng(7)
    ns = [int(v) for v in rng.integers(8200, 32768, 48)]
    probs = [var_problem(n, 1.1 + 0.8 * k / 47, seed=k) for k, n in enumerate(ns)]
    A = build(H, ctx, probs)
    x = rng.standard_normal(sum(ns))
    ys = []
    for _ in range(3):
        y = torch.zeros(sum(ns), dtype=torch.float64, device="cuda")
        A.toeplitz_matvec(dev(x), y)
        ys.append(y.cpu().numpy())
    A.close()
    assert all(np.array_equal(ys[0], y) for y in ys[1:])
    off = np.concatenate([[0], np.cumsum(ns)])
    for k in range(0, 48, 8):
        B = build(H, ctx, [probs[k]])
        yk = torch.zeros(ns[k], dtype=torch.float64, device="cuda")
        B.toeplitz_matvec(dev(x[off[k]:off[k + 1]]), yk)
        B.close()
        assert np.array_equal(yk.cpu().numpy(), ys[0][off[k]:off[k + 1]]), k
    for k in np.argsort(ns)[:2]:
        p, xk = probs[k], x[off[k]:off[k + 1]]
        ref = -O.residual_dd(p.alpha, p.nu, 1.0, p.d_plus, p.d_minus, xk, np.zeros(p.n))
        scale = np.abs(xk).max() * (1 + 4 * p.nu * max(p.d_plus.max(), p.d_minus.max()))
        assert np.max(np.abs(ys[0][off[k]:off[k + 1]] - ref)) <= 1e-13 * scale, k


@pytest.mark.parametrize("n,alpha,refine", [(1, 1.5, 0), (60, 1.5, 0), (1000, 1.2, 0), (1024, 1.5, 0),
                                            (1500, 1.8, 4), (4097, 1.8, 4)])
def test_factor_solve_fp64(H, ctx, n, alpha, refine):
    """FP64 HODLR LU + solve vs the oracle's refined dense solve: rel. error <= 1e-8.
    The truncation error of the factors grows like eps * cond(M); the stiff
    alpha = 1.8 cases take FP64 refinement sweeps with the exact residual."""
    p = var_problem(n, alpha, dt=1 / 16)
    A = build(H, ctx, [p], tol=1e-10, refine_max=refine, rtol=1e-12)
    A.factor()
    rng = np.random.default_rng(2)
    b = np.sin(7 * p.x) + 0.1 * rng.standard_normal(n)
    x = dev(b)
    A.solve(x, allow=(0, 2))
    ref = O.DenseSolver(alpha, n, p.nu, p.d_plus, p.d_minus).solve(b)
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 1e-8, err


@pytest.mark.parametrize("path,sizes", [("single", [(300, 1.3), (1024, 1.7), (77, 1.5)]),
                                        ("multi", [(1000, 1.3), (1000, 1.7), (1000, 1.5)]),
                                        ("multi", [(300, 1.3), (1024, 1.7), (77, 1.5), (1, 1.2), (2500, 1.9)])])
def test_batched_equals_separate(H, ctx, path, sizes):
    """A batch gives the same solutions as the problems run one by one, on the
    one-work-group-per-problem walk and on the multi-work-group schedule (same
    trees, and ragged trees of different depths merged step by step)."""
    import os
    os.environ["HODLR_FACTOR_PATH"] = path
    try:
        probs = [var_problem(n, a, seed=s) for s, (n, a) in enumerate(sizes)]
        A = build(H, ctx, probs)
        A.factor()
        rng = np.random.default_rng(3)
        bs = [rng.standard_normal(p.n) for p in probs]
        xb = dev(np.concatenate(bs))
        A.solve(xb)
        xb = xb.cpu().numpy()
        off = 0
        for p, b in zip(probs, bs):
            S = build(H, ctx, [p])
            S.factor()
            xs = dev(b)
            S.solve(xs)
            xs = xs.cpu().numpy()
            np.testing.assert_allclose(xb[off:off + p.n], xs, rtol=0, atol=1e-13 * np.abs(xs).max())
            off += p.n
    finally:
        del os.environ["HODLR_FACTOR_PATH"]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("alpha", [1.2, 1.8])
@pytest.mark.parametrize("gmres", [0, 8])
def test_mixed_precision_refined(H, ctx, prec, alpha, gmres):
    """Low-precision factors + FP64 refinement (exact residual), plain sweeps
    or GMRES-IR cycles of 8 iterations: rel. error <= 1e-10.  The low-precision
    path itself must get there (no FP64 fallback) except for BF16 factors at
    alpha = 1.8 with plain sweeps, where the contraction estimate exceeds one
    (the fallback then has to give the same accuracy)."""
    n = 3000
    p = var_problem(n, alpha, dt=1 / 256)
    A = build(H, ctx, [p], prec=prec, refine_max=8, rtol=1e-12, gmres_m=gmres)
    A.factor()
    b = np.cos(3 * p.x) * p.x
    x = dev(b)
    info = A.solve(x, allow=(0, 2))
    ref = O.DenseSolver(alpha, n, p.nu, p.d_plus, p.d_minus).solve(b)
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"{prec} alpha={alpha} gmres={gmres}: rel.err {err:.2e}, cycles {info.refine_iters}, "
          f"fallback {info.used_fallback}")
    assert err <= 1e-10, (err, info.refine_iters, info.rel_residual, info.used_fallback)
    if not (prec == "bf16" and alpha == 1.8 and gmres == 0):
        assert info.used_fallback == 0, (prec, alpha, gmres, info.refine_iters)


@pytest.mark.parametrize("gmres", [0, 4])
def test_time_steps_checked_against_solves(H, ctx, gmres):
    """The graph time loop (three sweeps a step, plain or GMRES-IR, FP32
    factors, two problems of different sizes) equals step-by-step refined
    solves against the oracle within 1e-10, reports no fallback, and its worst
    per-step correction is below the target."""
    probs = [var_problem(2500, 1.7, dt=1 / 64, seed=3), var_problem(700, 1.3, dt=1 / 64, seed=4)]
    A = build(H, ctx, probs, prec="fp32", refine_max=3, rtol=1e-10, gmres_m=gmres)
    A.factor()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        A.ctx = H.Context(stream)
        u = dev(np.concatenate([p.u0 for p in probs]))
        info = A.time_steps(u, None, 0.0, 5)
        stream.synchronize()
    assert info.used_fallback == 0 and info.rel_correction <= 1e-10, (info.used_fallback, info.rel_correction)
    off = 0
    for p in probs:
        ref = O.euler_1d(p, steps=5)
        got = u.cpu().numpy()[off:off + p.n]
        off += p.n
        assert np.linalg.norm(got - ref) <= 1e-10 * np.linalg.norm(ref)


def test_time_steps_plain_config(H, ctx):
    """Workload 'plain_1d' (N=1024, alpha=1.5, 16 implicit Euler steps, FP64 factors).
    eps = 1e-10 leaves ~1e-9 per step, which accumulates over 16 steps; one FP64
    refinement sweep per step (exact residual) removes it."""
    p = W.plain_1d()
    A = build(H, ctx, [p], tol=1e-10, refine_max=1, rtol=1e-12)
    A.factor()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        c2 = H.Context(stream)
        A.ctx = c2
        u = dev(p.u0)
        A.time_steps(u, None, 0.0, p.steps, allow=(0, 2))
        stream.synchronize()
    ref = O.euler_1d(p)
    err = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 1e-8, err


@pytest.mark.parametrize("n,alpha", [(700, 1.4), (2049, 1.8)])
def test_factor_paths_agree(H, ctx, n, alpha):
    """The one-work-group-per-problem walk and the multi-work-group schedule
    carry out the same factorisation (different summation orders).  Without
    refinement the error of the factors is bounded by about eps * cond(M) and,
    in the Gram-based recompression, by sqrt(u) times the norm of each updated
    block; the stiff alpha = 1.8 case (cond ~ 1e5) therefore takes FP64
    refinement sweeps with the exact residual."""
    import os
    p = var_problem(n, alpha, dt=1 / 32)
    b = np.cos(5 * p.x) + p.x
    sols = []
    for path in ("single", "multi"):
        os.environ["HODLR_FACTOR_PATH"] = path
        try:
            A = build(H, ctx, [p], tol=1e-10, refine_max=0 if alpha < 1.5 else 3, rtol=1e-12)
            A.factor()
            x = dev(b)
            A.solve(x, allow=(0, 2))
            sols.append(x.cpu().numpy())
        finally:
            del os.environ["HODLR_FACTOR_PATH"]
    ref = O.DenseSolver(alpha, n, p.nu, p.d_plus, p.d_minus).solve(b)
    errs = [np.linalg.norm(s - ref) / np.linalg.norm(ref) for s in sols]
    assert max(errs) <= 1e-8, errs     # both within the truncation error of eps = 1e-10
    # they differ only where Gram rounding moves a rank decision at the margin
    assert np.linalg.norm(sols[0] - sols[1]) / np.linalg.norm(ref) <= 1e-8


def test_ragged_batch_time_steps(H, ctx):
    """Ragged batch (the batched workload's recipe at small sizes: N log-uniform,
    alpha uniform in (1.1, 1.9), one operator per problem): every problem's
    implicit Euler trajectory matches the oracle's, from one batched factor and
    one batched time-step loop."""
    probs = W.batched_1d(count=10, nmin=100, nmax=6000, steps=6)
    A = build(H, ctx, probs, tol=1e-10, refine_max=2, rtol=1e-12)
    A.factor()
    u = dev(np.concatenate([p.u0 for p in probs]))
    f = dev(np.concatenate([p.f for p in probs]))
    A.time_steps(u, f, probs[0].dt, probs[0].steps, allow=(0, 2))
    u = u.cpu().numpy()
    off = 0
    for p in probs:
        ref = O.euler_1d(p)
        err = np.linalg.norm(u[off:off + p.n] - ref) / np.linalg.norm(ref)
        assert err <= 1e-9, (p.name, err)
        off += p.n


def test_autotune_then_factor(H, ctx):
    """The autotuner picks launch shapes from its candidate set and the
    factorisation with them solves as accurately as with the defaults (two
    FP64 refinement sweeps with the exact residual, as for the other cases whose
    condition number exceeds about 1e4)."""
    p = var_problem(3000, 1.5, dt=1 / 64)
    b = np.cos(4 * p.x) + p.x
    A = build(H, ctx, [p, p], tol=1e-10, refine_max=2, rtol=1e-12)
    t = A.autotune()
    assert t.core_threads in (256, 512) and t.leaf_threads in (256, 512) and t.gram_rows in (128, 256, 512)
    assert t.fuse_rows in (0, 128, 256, 512, 1024)
    assert t.factor_ms > 0
    A.factor()
    x = dev(np.concatenate([b, b]))
    A.solve(x, allow=(0, 2))
    ref = O.DenseSolver(1.5, p.n, p.nu, p.d_plus, p.d_minus).solve(b)
    xs = x.cpu().numpy()
    for k in range(2):
        assert np.linalg.norm(xs[k * p.n:(k + 1) * p.n] - ref) / np.linalg.norm(ref) <= 1e-9
    B = build(H, ctx, [p, p], tol=1e-10, refine_max=2, rtol=1e-12)      # same tree signature: tuned shapes reused
    B.factor()
    y = dev(np.concatenate([b, b]))
    B.solve(y, allow=(0, 2))
    assert np.linalg.norm(y.cpu().numpy() - xs) <= 1e-12 * np.linalg.norm(xs)


def test_fused_and_split_node_steps_agree(H, ctx):
    """Phase A of a node as fused single-work-group kernels (Grams, core and
    forms in one launch) and as the split multi-work-group kernels compute the
    same factors up to the rounding order of the Gram sums; a ragged batch
    exercises both kinds of step in one schedule."""
    probs = [var_problem(3000, 1.3, dt=1 / 64), var_problem(1700, 1.6, dt=1 / 64)]
    rng = np.random.default_rng(5)
    bs = [np.sin(3 * p.x) + 0.1 * rng.standard_normal(p.n) for p in probs]
    refs = [O.DenseSolver(p.alpha, p.n, p.nu, p.d_plus, p.d_minus).solve(b) for p, b in zip(probs, bs)]
    sols = []
    for fuse in (0, 1024, 256):
        A = build(H, ctx, probs, tol=1e-10, refine_max=2, rtol=1e-12)
        A.set_tuning(fuse_rows=fuse)
        A.factor()
        x = dev(np.concatenate(bs))
        A.solve(x, allow=(0, 2))
        xs = x.cpu().numpy()
        sols.append(xs)
        off = 0
        for p, ref in zip(probs, refs):
            err = np.linalg.norm(xs[off:off + p.n] - ref) / np.linalg.norm(ref)
            assert err <= 1e-9, (fuse, p.n, err)
            off += p.n
    for s in sols[1:]:
        assert np.linalg.norm(s - sols[0]) <= 1e-9 * np.linalg.norm(sols[0])


def test_time_dependent_coefficients(H, ctx):
    """Coefficients d+(x, t), d-(x, t) that change every step: the compressed
    operator is rebuilt in place and factored again each step (a ragged batch
    of two problems), and the trajectory matches the oracle's per-step dense
    solves.  Solving between the update and the new factorisation is refused."""
    probs = [var_problem(1500, 1.4, dt=1 / 32), var_problem(900, 1.7, dt=1 / 32, seed=1)]
    steps = 6
    A = build(H, ctx, probs, tol=1e-10, refine_max=3, rtol=1e-12)
    u = dev(np.concatenate([p.u0 for p in probs]))
    for m in range(1, steps + 1):
        coefs = [W.timedep_coefficients(p, m * p.dt) for p in probs]
        A.update_coefficients([H.operator_dict(p.n, p.alpha, p.dt, p.h, dev(dp), dev(dm), 1.0)
                               for p, (dp, dm) in zip(probs, coefs)])
        if m == 1:
            with pytest.raises(H.HodlrError):
                A.solve(u.clone())
        A.factor()
        A.solve(u, allow=(0, 2))          # f = 0: the right-hand side is u^(m-1)
    us = u.cpu().numpy()
    off = 0
    for p in probs:
        ref = O.euler_1d_varying(p, lambda t, p=p: W.timedep_coefficients(p, t), steps=steps)
        err = np.linalg.norm(us[off:off + p.n] - ref) / np.linalg.norm(ref)
        assert err <= 1e-9, (p.n, err)
        off += p.n
    with pytest.raises(H.HodlrError):      # n must not change
        A.update_coefficients([H.operator_dict(p.n + 1, p.alpha, p.dt, p.h, dev(np.ones(p.n + 1)),
                                               dev(np.ones(p.n + 1)), 1.0) for p in probs])


def test_pooled_blocks_give_identical_results(H, ctx):
    """A destroyed matrix's device blocks go to the library's pool and a new
    matrix of the same shape takes them (stale contents included): building,
    factoring and solving the same problems three times in a row, FP32 and
    FP64 storage interleaved, gives the same bits every time, and the pooled
    build holds the same device bytes."""
    probs = [var_problem(3000, 1.35), var_problem(1500, 1.7, seed=3)]
    b = np.concatenate([np.sin(3 * p.x) + p.x for p in probs])
    seen = {}
    for rep in range(3):
        for prec in ("fp32", "fp64"):
            A = build(H, ctx, probs, tol=1e-10, prec=prec, refine_max=2, rtol=1e-12)
            A.factor()
            x = dev(b)
            A.solve(x, allow=(0, 2))
            got = (x.cpu().numpy(), A.info().bytes_device)
            A.close()
            if prec in seen:
                assert np.array_equal(got[0], seen[prec][0]), (rep, prec)
                assert got[1] == seen[prec][1]
            else:
                seen[prec] = got
    ref = np.concatenate([O.DenseSolver(p.alpha, p.n, p.nu, p.d_plus, p.d_minus).solve(r)
                          for p, r in zip(probs, np.split(b, [probs[0].n]))])
    for prec in ("fp32", "fp64"):
        assert np.linalg.norm(seen[prec][0] - ref) <= 1e-9 * np.linalg.norm(ref), prec


def test_workspace_build_equals_library_allocated(H, ctx):
    """A batch built with hodlr_build_ws into a torch-allocated workspace (the
    binding's default) that starts filled with NaN bytes gives the same exact
    product, factors and refined
    solution, bit for bit, as one the library allocates (hodlr_build); a
    workspace one page short of hodlr_workspace_size is refused with
    HODLR_EINVAL naming argument 6."""
    import ctypes as C
    from paper_1804_05522_amd import hodlr as HB
    probs = [var_problem(3000, 1.5, seed=1), var_problem(777, 1.8, seed=2)]
    ops = [H.operator_dict(p.n, p.alpha, p.dt, p.h, dev(p.d_plus), dev(p.d_minus)) for p in probs]
    opts = H.default_opts(tol=1e-10, prec="fp32", refine_max=4, rtol=1e-12)
    n = sum(p.n for p in probs)
    rng = np.random.default_rng(5)
    b = dev(rng.standard_normal(n))
    outs = []
    import os
    for ws in (False, True):
        os.environ["HODLR_POISON"] = "1" if ws else "0"   # the workspace starts as NaN bytes
        try:
            A = H.HodlrMatrix(ctx, ops, opts, workspace=ws)
        finally:
            os.environ.pop("HODLR_POISON", None)
        y = torch.zeros(n, dtype=torch.float64, device="cuda")
        A.toeplitz_matvec(b, y)
        A.factor()
        x = b.clone()
        info = A.solve(x)
        torch.cuda.synchronize()
        assert info.used_fallback == 0
        outs.append((y.cpu().numpy(), x.cpu().numpy(), A.info().max_rank_factors))
        A.close()
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])
    assert outs[0][2] == outs[1][2]
    L = H.lib()
    arr = H.HodlrMatrix._op_array(ops)
    need = C.c_size_t()
    assert L.hodlr_workspace_size(arr, len(ops), C.byref(opts), C.byref(need)) == 0
    short = torch.empty(need.value - 4096, dtype=torch.uint8, device="cuda")
    h = C.c_void_p()
    st = L.hodlr_build_ws(ctx.h, arr, len(ops), C.byref(opts), C.c_void_p(short.data_ptr()), need.value - 4096,
                          C.byref(h))
    assert st == HB.HODLR_EINVAL and L.hodlr_last_arg(ctx.h) == 6 and not h.value
