"""CPU oracle for the learned warm start's network (test infrastructure).

TEST INFRASTRUCTURE ONLY; see ``oracle/__init__.py``.

The network that predicts u_{k+1} from u_k (a production pattern of the
build, not part of the paper) is four 3x3 convolutions with zero padding
(zero = the absorbing boundary of eq. (fde_FD)), channels 1 -> C -> C -> C -> 1,
ReLU after the first three, and a residual output
    u_{k+1} ~ u_k + net(u_k).
Loss: mean squared error.  Optimiser: Adam (Kingma & Ba, 2015).

Everything here is FP64 and written with explicit loops over the nine taps,
so each formula can be read off directly:
    y[o, i, j] = b[o] + sum_c sum_{p,q in {-1,0,1}} w[o, c, p+1, q+1] x[c, i+p, j+q]
(cross-correlation, x = 0 outside the image).
"""
from __future__ import annotations

import numpy as np


def _pad(x):
    return np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))


def conv3x3(x, w, b):
    """x: (n, c, h, w); w: (o, c, 3, 3); b: (o,) -> (n, o, h, w)."""
    n, c, H, W = x.shape
    xp = _pad(x)
    y = np.zeros((n, w.shape[0], H, W))
    for p in range(3):
        for q in range(3):
            patch = xp[:, :, p:p + H, q:q + W]            # (n, c, H, W)
            y += np.einsum("nchw,oc->nohw", patch, w[:, :, p, q])
    return y + b[None, :, None, None]


def conv3x3_backward(x, w, gy):
    """Gradients of conv3x3 wrt x, w and b given dL/dy."""
    n, c, H, W = x.shape
    xp = _pad(x)
    gw = np.zeros_like(w)
    gxp = np.zeros_like(xp)
    for p in range(3):
        for q in range(3):
            patch = xp[:, :, p:p + H, q:q + W]
            gw[:, :, p, q] = np.einsum("nohw,nchw->oc", gy, patch)
            gxp[:, :, p:p + H, q:q + W] += np.einsum("nohw,oc->nchw", gy, w[:, :, p, q])
    gb = gy.sum(axis=(0, 2, 3))
    return gxp[:, :, 1:-1, 1:-1], gw, gb


def init_params(rng, channels=32, scale_last=1e-2):
    """He-style initialisation; the last layer starts small (prediction ~ u_k)."""
    shapes = [(channels, 1), (channels, channels), (channels, channels), (1, channels)]
    params = []
    for li, (o, c) in enumerate(shapes):
        std = np.sqrt(2.0 / (9 * c))
        if li == len(shapes) - 1:
            std *= scale_last
        params.append([rng.normal(0.0, std, (o, c, 3, 3)), np.zeros(o)])
    return params


def forward(params, u):
    """u: (n, 1, h, w) -> prediction and the activations needed for backward."""
    acts = [u]
    h = u
    pre = []
    for li, (w, b) in enumerate(params):
        z = conv3x3(h, w, b)
        pre.append(z)
        h = np.maximum(z, 0.0) if li < len(params) - 1 else z
        acts.append(h)
    return u + h, acts, pre


def loss_and_grads(params, u, target):
    """MSE loss mean((pred - target)^2) and its gradients for every parameter."""
    pred, acts, pre = forward(params, u)
    diff = pred - target
    loss = float(np.mean(diff * diff))
    g = 2.0 * diff / diff.size
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        w, _ = params[li]
        if li < len(params) - 1:
            g = g * (pre[li] > 0)
        gx, gw, gb = conv3x3_backward(acts[li], w, g)
        grads[li] = [gw, gb]
        g = gx
    return loss, grads


class Adam:
    """Adam: m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
    p <- p - lr * mhat / (sqrt(vhat) + eps), with bias-corrected mhat, vhat."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [[np.zeros_like(a) for a in p] for p in params]
        self.v = [[np.zeros_like(a) for a in p] for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        c1 = 1 - self.b1 ** self.t
        c2 = 1 - self.b2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            for k in range(len(p)):
                m[k] = self.b1 * m[k] + (1 - self.b1) * g[k]
                v[k] = self.b2 * v[k] + (1 - self.b2) * g[k] * g[k]
                p[k] = p[k] - self.lr * (m[k] / c1) / (np.sqrt(v[k] / c2) + self.eps)
        return params
