"""The no-allocation exact product (static device scratch) against the
product with the handle's own scratch: same kernels, one column a launch, so
the results must agree bit for bit.  Two calls in a row, the second on a
smaller matrix (the static array keeps the first call's contents), then a
matrix whose packed scratch exceeds the static maximum is refused."""
import numpy as np
import pytest

import workloads as W

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


def build(H, ctx, probs, kinds=None):
    kinds = kinds or [0] * len(probs)
    ops = [H.operator_dict(p.n, p.alpha, p.dt, p.h, dev(p.d_plus), dev(p.d_minus), discretization=k)
           for p, k in zip(probs, kinds)]
    return H.HodlrMatrix(ctx, ops, H.default_opts(tol=1e-10))


def compare(H, ctx, stream, A, n, nrhs, seed):
    rng = np.random.default_rng(seed)
    x = dev(rng.standard_normal((nrhs, n)))
    y_ref = torch.full((nrhs, n), np.nan, dtype=torch.float64, device="cuda")
    y_new = torch.full((nrhs, n), np.nan, dtype=torch.float64, device="cuda")
    A.toeplitz_matvec(x, y_ref, nrhs=nrhs)
    A.toeplitz_matvec_noalloc(x, y_new, nrhs=nrhs)
    stream.synchronize()
    a, b = y_ref.cpu().numpy(), y_new.cpu().numpy()
    assert np.all(np.isfinite(b))
    assert np.array_equal(a, b), float(np.max(np.abs(a - b)))


def test_noalloc_product_equals_the_product(H):
    stream = torch.cuda.Stream()
    ctx = H.Context(stream)
    with torch.cuda.stream(stream):
        big = [W.var_1d(1.2, n=65536), W.var_1d(1.8, n=65536)]    # 2 x 2 x 2^17 complex: 8 MiB of 16
        A = build(H, ctx, big)
        compare(H, ctx, stream, A, 2 * 65536, 3, 1)
        A.close()
        small = [W.plain_1d(), W.var_1d(1.5, n=3000)]              # second call: smaller input,
        B = build(H, ctx, small, kinds=[H.FDE_FD, H.FDE_FE])      # one finite-element operator
        compare(H, ctx, stream, B, 1024 + 3000, 2, 2)
        B.close()
        over = [W.var_1d(1.4, n=300000)]                           # 2 x 2^20 complex: 32 MiB
        Cm = build(H, ctx, over)
        x = torch.zeros(300000, dtype=torch.float64, device="cuda")
        y = torch.zeros(300000, dtype=torch.float64, device="cuda")
        with pytest.raises(H.HodlrError):
            Cm.toeplitz_matvec_noalloc(x, y)
        Cm.close()
    ctx.close()
