"""GPU parity of the learned warm start's network (forward, gradients, Adam)
against the CPU oracle, through the C ABI."""
import numpy as np
import pytest

from oracle import convnet as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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


def setup(seed, n=2, h=20, w=24, scale_last=1.0):
    rng = np.random.default_rng(seed)
    params = O.init_params(rng, channels=32, scale_last=scale_last)
    for wb in params:                      # nonzero biases exercise the bias paths
        wb[1] = 0.05 * rng.standard_normal(wb[1].shape)
    u = rng.standard_normal((n, 1, h, w))
    target = u + 0.1 * rng.standard_normal((n, 1, h, w))
    # FP32 inputs as the GPU sees them
    params = [[np.float32(a).astype(np.float64) for a in wb] for wb in params]
    return params, np.float32(u).astype(np.float64), np.float32(target).astype(np.float64)


def gpu(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device="cuda")


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300)


@pytest.mark.parametrize("shape", [(2, 20, 24), (1, 33, 7), (3, 64, 64)])
def test_forward_fp32_matches_oracle(H, ctx, shape):
    params, u, _ = setup(1, *shape)
    net = H.ConvNet(ctx, bf16=False, max_pixels=int(np.prod(shape)))
    net.set_params(params)
    pred = torch.zeros(shape, dtype=torch.float32, device="cuda")
    net.forward(gpu(u[:, 0]), pred)
    ref, _, _ = O.forward(params, u)
    assert rel(pred.cpu().numpy(), ref[:, 0]) < 1e-5


def test_grads_fp32_match_oracle(H, ctx):
    params, u, target = setup(2)
    net = H.ConvNet(ctx, bf16=False, max_pixels=u.size)
    net.set_params(params)
    loss = net.train_step(gpu(u[:, 0]), gpu(target[:, 0]), margin=0, lr=0.0, update=False)
    rloss, rgrads = O.loss_and_grads(params, u, target)
    assert abs(loss - rloss) <= 1e-5 * rloss
    g = H.ConvNet.unflatten(net.get_grads())
    for li in range(4):
        for k in range(2):
            assert rel(g[li][k], rgrads[li][k]) < 1e-4, (li, k, rel(g[li][k], rgrads[li][k]))


def test_bf16_matrix_cores_match_oracle(H, ctx):
    """BF16 activations on the matrix cores: forward and gradients within the
    precision of BF16 storage (8 significant bits)."""
    params, u, target = setup(3, n=2, h=64, w=64)
    net = H.ConvNet(ctx, bf16=True, max_pixels=u.size)
    net.set_params(params)
    pred = torch.zeros(u[:, 0].shape, dtype=torch.float32, device="cuda")
    net.forward(gpu(u[:, 0]), pred)
    ref, _, _ = O.forward(params, u)
    # compare the network part (the residual connection is exact)
    assert rel(pred.cpu().numpy() - u[:, 0], ref[:, 0] - u[:, 0]) < 2e-2
    net.train_step(gpu(u[:, 0]), gpu(target[:, 0]), margin=0, lr=0.0, update=False)
    _, rgrads = O.loss_and_grads(params, u, target)
    g = H.ConvNet.unflatten(net.get_grads())
    for li in range(4):
        assert rel(g[li][0], rgrads[li][0]) < 5e-2, (li, rel(g[li][0], rgrads[li][0]))


def test_margin_excludes_border(H, ctx):
    """Pixels within the margin carry no loss: changing the target there changes nothing."""
    params, u, target = setup(4, n=1, h=16, w=16)
    net = H.ConvNet(ctx, bf16=False, max_pixels=u.size)
    net.set_params(params)
    l1 = net.train_step(gpu(u[:, 0]), gpu(target[:, 0]), margin=3, lr=0.0, update=False)
    t2 = target.copy()
    t2[:, :, :3, :] += 5.0
    t2[:, :, :, -3:] -= 5.0
    l2 = net.train_step(gpu(u[:, 0]), gpu(t2[:, 0]), margin=3, lr=0.0, update=False)
    assert abs(l1 - l2) <= 1e-6 * l1
    pred, _, _ = O.forward(params, u)
    inner = (pred - target)[:, :, 3:-3, 3:-3]
    assert abs(l1 - np.mean(inner ** 2)) <= 1e-5 * l1


def test_adam_steps_match_oracle(H, ctx):
    params, u, target = setup(5)
    net = H.ConvNet(ctx, bf16=False, max_pixels=u.size)
    net.set_params(params)
    ref = [[a.copy() for a in wb] for wb in params]
    opt = O.Adam(ref, lr=1e-3)
    for _ in range(3):
        net.train_step(gpu(u[:, 0]), gpu(target[:, 0]), margin=0, lr=1e-3, update=True)
        _, g = O.loss_and_grads(ref, u, target)
        ref = opt.step(ref, g)
    got = H.ConvNet.unflatten(net.get_params())
    for li in range(4):
        for k in range(2):
            # each Adam step moves a weight by about lr; allow 1e-3 of that
            assert np.max(np.abs(got[li][k] - ref[li][k])) < 3e-6, (li, k)
