"""Forward error of the benchmark's 1D configuration against stored oracle
trajectories (tests/golden/make_var1d.py: dense LU of M, every step refined
with the double-double residual, so exact to about unit roundoff).

The GPU side runs exactly what the benchmark times: both alphas as one batch,
FP32 factors, factorisation launch shapes from the autotuner, the time loop
replayed from its HIP graph on a non-default stream, three FP64 refinement
sweeps a step with the exact Toeplitz residual, each step's correction checked
on the device.  At every stored step both problems must satisfy
  ||u - u_ref||_2 <= 1e-10 ||u_ref||_2  and  max|u - u_ref| <= 1e-10 max|u_ref|,
and the mixed path must be what produced them (no FP64 fallback)."""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-10


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1804_05522_amd as H
    H.lib()
    return H


def run_against_golden(H, n, sweeps=3):
    path = os.path.join(GOLDEN, f"var1d_n{n}.npz")
    g = np.load(path)
    alphas = [float(a) for a in g["alphas"]]
    stored = [int(s) for s in g["steps"]]
    probs = [W.var_1d(a, n=n) for a in alphas]
    stream = torch.cuda.Stream()
    ctx = H.Context(stream)
    with torch.cuda.stream(stream):
        ops = [H.operator_dict(p.n, p.alpha, p.dt, p.h, dev(p.d_plus), dev(p.d_minus)) for p in probs]
        At = H.HodlrMatrix(ctx, ops, H.default_opts(tol=1e-10, prec="fp32"))
        At.autotune()
        At.close()
        A = H.HodlrMatrix(ctx, ops, H.default_opts(tol=1e-10, prec="fp32", refine_max=sweeps, rtol=TOL))
        A.factor(allow=(0, 3))
        u = dev(np.concatenate([p.u0 for p in probs]))
        f = dev(np.concatenate([p.f for p in probs]))
        done = 0
        report = []
        for j, m in enumerate(stored):
            info = A.time_steps(u, f, probs[0].dt, m - done)
            done = m
            stream.synchronize()
            assert not info.used_fallback, (n, m, "a step fell back to the FP64 factors")
            assert info.rel_correction <= TOL, (n, m, info.rel_correction)
            uh = u.cpu().numpy()
            for k, a in enumerate(alphas):
                ug = uh[k * n:(k + 1) * n]
                ref = g[f"u_a{a}"][j]
                e2 = np.linalg.norm(ug - ref) / np.linalg.norm(ref)
                einf = np.max(np.abs(ug - ref)) / np.max(np.abs(ref))
                report.append((m, a, e2, einf))
                assert e2 <= TOL and einf <= TOL, (n, m, a, e2, einf)
        A.close()
    ctx.close()
    for m, a, e2, einf in report:
        print(f"N={n} step {m} alpha={a}: rel.err 2-norm {e2:.2e}, max-norm {einf:.2e}")


def test_var1d_n16384_whole_trajectory(H):
    """All 256 steps at N = 16384, compared at steps 1, 2, 4, ..., 256."""
    run_against_golden(H, 16384)


def test_var1d_n65536_first_steps(H):
    """The benchmark's size, N = 65536: steps 1 to 4."""
    if not os.path.exists(os.path.join(GOLDEN, "var1d_n65536.npz")):
        pytest.skip("golden trajectory at N=65536 not generated")
    run_against_golden(H, 65536)
