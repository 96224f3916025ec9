"""Learned warm start on the GPU: the network is trained on trajectories that
the HODLR Sylvester solver itself generates, its prediction of the next step is
compressed and handed to the per-step solver as the first iterate, and the
solver's exact residual decides whether the guess is used.  Every warm step is
checked against the cold step and against the oracle's Bartels-Stewart
solution; the ADI step counts of the two starts are reported side by side."""
import numpy as np
import pytest

import workloads as W
from oracle import convnet as OC
from oracle import fde2d as O2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N = 256
STEPS = 6


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
def setup(H):
    ctx = H.Context()
    p0 = W.learned_2d(n=N, seed=0)
    opx = H.operator_dict(N, p0.alpha_x, p0.dt, p0.hx, dev(p0.dxp), dev(p0.dxm), 0.5)
    opy = H.operator_dict(N, p0.alpha_y, p0.dt, p0.hy, dev(p0.dyp), dev(p0.dym), 0.5)
    P = H.Fde2dPlan(ctx, opx, opy, H.default_opts(tol=1e-12, prec="fp64", leaf=64), tol=1e-8)
    zero = (torch.zeros((0, N), dtype=torch.float64, device="cuda"),) * 2

    def field(lr):
        f = torch.zeros((N, N), dtype=torch.float32, device="cuda")
        P.to_field(lr, f)
        return f

    def trajectory(seed):
        p = W.learned_2d(n=N, seed=seed, steps=STEPS)
        cur = (dev(p.u0.Z.T.copy()), dev(p.u0.W.T.copy()))
        lrs, fields, adi = [cur], [field(cur)], []
        for _ in range(STEPS):
            out = newout()
            r, info = P.step(cur, zero, p.dt, out, allow=(0, 2))
            cur = (out[0][:r].contiguous(), out[1][:r].contiguous())
            lrs.append(cur)
            fields.append(field(cur))
            adi.append(info.refine_iters)
        return p, lrs, fields, adi

    trajs = [trajectory(s) for s in range(5)]
    return ctx, P, zero, trajs


def newout():
    return (torch.zeros((64, N), dtype=torch.float64, device="cuda"),
            torch.zeros((64, N), dtype=torch.float64, device="cuda"))


def dense(lr):
    return lr[0].cpu().numpy().T @ lr[1].cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def train(H, ctx, trajs, iters=600):
    """BF16 network trained on (u_k, u_{k+1}) pairs of the first trajectories;
    returns it with its loss on a fixed batch of training pairs before and
    after training."""
    net = H.ConvNet(ctx, bf16=True, max_pixels=4 * N * N)
    net.set_params(OC.init_params(np.random.default_rng(0), 32))
    pairs = [(t[2][k], t[2][k + 1]) for t in trajs for k in range(STEPS)]
    fixed = (torch.stack([pairs[i][0] for i in (0, 7, 14, 21)]),
             torch.stack([pairs[i][1] for i in (0, 7, 14, 21)]))
    before = net.train_step(*fixed, margin=0, lr=0.0, update=False)
    rng = np.random.default_rng(1)
    for it in range(iters):
        idx = rng.choice(len(pairs), 4, replace=False)
        u = torch.stack([pairs[i][0] for i in idx])
        tg = torch.stack([pairs[i][1] for i in idx])
        net.train_step(u, tg, margin=0, lr=1e-3 if it < 0.7 * iters else 2e-4)
    after = net.train_step(*fixed, margin=0, lr=0.0, update=False)
    return net, before, after


def test_trajectories_match_oracle(setup):
    """The training data: HODLR trajectories equal the oracle's Bartels-Stewart steps."""
    _, _, _, trajs = setup
    p, lrs, _, _ = trajs[0]
    st = O2.SylvesterStepper(p)
    U = p.u0.dense()
    for k in range(STEPS):
        U = st.step(U, np.zeros_like(U))
        assert rel(dense(lrs[k + 1]), U) <= 1e-7, k


def test_learned_warm_start(H, setup):
    """The trained network predicts the next step better than the identity
    guess; every warm step, used or rejected, matches the cold step and the
    oracle; the ADI steps of both starts are reported."""
    ctx, P, zero, trajs = setup
    net, before, after = train(H, ctx, trajs[:4])
    p, lrs, fields, adi_cold = trajs[4]          # held out
    st = O2.SylvesterStepper(p)
    pred = torch.zeros((1, N, N), dtype=torch.float32, device="cuda")
    e_net, e_id, adi_warm, used = [], [], [], 0
    for k in range(STEPS):
        net.forward(fields[k][None], pred)
        e_net.append(float(torch.linalg.norm(pred[0] - fields[k + 1]) / torch.linalg.norm(fields[k + 1])))
        e_id.append(float(torch.linalg.norm(fields[k] - fields[k + 1]) / torch.linalg.norm(fields[k + 1])))
        g = (torch.zeros((10, N), dtype=torch.float64, device="cuda"),
             torch.zeros((10, N), dtype=torch.float64, device="cuda"))
        rg = P.compress_field(pred[0].contiguous(), 1e-2, g, seed=k + 1)
        out = newout()
        r, info = P.step(lrs[k], zero, p.dt, out, allow=(0, 2), guess=g, guess_rank=rg)
        X = dense((out[0][:r], out[1][:r]))
        assert rel(X, dense(lrs[k + 1])) <= 1e-7, (k, info.used_fallback)
        ref = st.step(dense(lrs[k]), np.zeros((N, N)))
        assert rel(X, ref) <= 1e-7, k
        adi_warm.append(info.refine_iters)
        used += 1 - info.used_fallback
    print(f"\ntraining loss {before:.3e} -> {after:.3e}; held-out one-step error: net {np.round(e_net, 3)} "
          f"identity {np.round(e_id, 3)}; ADI steps cold {adi_cold} warm {adi_warm}; guesses used {used}/{STEPS}")
    assert after < 0.7 * before
    assert np.mean(e_net) < np.mean(e_id)
    # a guess is used only when its residual saves at least one block of
    # shifts, so no warm step takes more ADI steps than the cold one
    assert all(w <= c for w, c in zip(adi_warm, adi_cold)), (adi_warm, adi_cold)


def test_exact_guess_cuts_adi_steps(H, setup):
    """With the solution itself as the guess (the step solved by a plan at a
    thousandfold tighter tolerance, so that its residual lies well below the
    stopping level) a block or two of four shifts confirm it, against a full
    sweep plus a confirming block from the zero guess."""
    ctx, P, zero, trajs = setup
    p, lrs, _, adi_cold = trajs[1]
    opx = H.operator_dict(N, p.alpha_x, p.dt, p.hx, dev(p.dxp), dev(p.dxm), 0.5)
    opy = H.operator_dict(N, p.alpha_y, p.dt, p.hy, dev(p.dyp), dev(p.dym), 0.5)
    Pt = H.Fde2dPlan(ctx, opx, opy, H.default_opts(tol=1e-14, prec="fp64", leaf=64), tol=1e-11)
    try:
        for k in range(2):
            ex = newout()
            re, _ = Pt.step(lrs[k], zero, p.dt, ex, allow=(0, 2))
            out = newout()
            r, info = P.step(lrs[k], zero, p.dt, out, allow=(0, 2), guess=(ex[0][:re], ex[1][:re]), guess_rank=re)
            assert info.used_fallback == 0
            assert info.refine_iters <= 8 and info.refine_iters < adi_cold[k], (info.refine_iters, adi_cold[k])
            assert rel(dense((out[0][:r], out[1][:r])), dense(lrs[k + 1])) <= 1e-7
    finally:
        Pt.close()


def test_bad_guess_falls_back_to_plain_solve(H, setup):
    """An untrained network with a large last layer predicts garbage: its
    residual exceeds that of the zero guess, the solver takes the plain path
    and returns the cold step's result bit for bit."""
    ctx, P, zero, trajs = setup
    p, lrs, fields, _ = trajs[2]
    net = H.ConvNet(ctx, bf16=False, max_pixels=N * N)
    net.set_params(OC.init_params(np.random.default_rng(7), 32, scale_last=50.0))
    pred = torch.zeros((1, N, N), dtype=torch.float32, device="cuda")
    net.forward(fields[0][None], pred)
    g = (torch.zeros((10, N), dtype=torch.float64, device="cuda"),
         torch.zeros((10, N), dtype=torch.float64, device="cuda"))
    rg = P.compress_field(pred[0].contiguous(), 1e-2, g, seed=3)
    out = newout()
    r, info = P.step(lrs[0], zero, p.dt, out, allow=(0, 2), guess=g, guess_rank=rg)
    assert info.used_fallback == 1
    assert torch.equal(out[0][:r], lrs[1][0]) and torch.equal(out[1][:r], lrs[1][1])
