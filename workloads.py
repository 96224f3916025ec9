"""Seeded synthetic inputs for the fractional-diffusion workloads.

This module is shared by the CPU oracle and the GPU path.  It produces only
*inputs* of the problems (grids, diffusion-coefficient samples, initial data,
source terms, parameters of each workload) and holds none of the method's
arithmetic: no Grunwald-Letnikov weights, no matrices, no solves.

Grid convention (Sec. 2.2.1, eq. (part)): N interior points x_i = L + i*h,
i = 1..N, h = (R - L)/(N + 1), absorbing boundary (u = 0 outside (L, R)).

Workload recipes (the shapes of the paper's experiments; inputs the paper
does not state are the choices written out below):

* ``plain_1d``   N=1024, alpha=1.5, d+=d-=1, dt=1/16, 16 steps,
                 u0=x^2(1-x)^2, f=0.
* ``var_1d``     N=65536, alpha in {1.2, 1.8}, d+=1+x^2, d-=1+(1-x)^2,
                 dt=1/256 (T=1), 256 steps, u0=x^2(1-x)^2,
                 f = sum of 8 seeded Gaussians (time independent).
* ``batched_1d`` 256 problems, N log-uniform in [2048, 32768],
                 alpha~U(1.1,1.9), d+=d-=1+a sin(pi k x), a~U(0,0.5),
                 k~U{1..4}, dt=1/64, 64 steps, u0=x^2(1-x)^2, 8-Gaussian f.
* ``fd_2d``      4096 x 4096 grid on [0,1]^2, alpha1=1.3, alpha2=1.7,
                 coefficients of eq. (coeff_es) read as d_{1,+-}(x),
                 d_{2,+-}(y), U0=0, rank-4 separable Gaussian source, dt=1/64,
                 64 steps.
* ``learned_2d`` 2048 x 2048, alpha1=1.4, alpha2=1.6, d+-=1, f=0, dt=1/64,
                 initial conditions = sums of 8 separable Gaussians.
* ``fe_1d``      finite elements (P1 hats) in 1D: N=4096, alpha=1.3,
                 d+=d-=1 (constant, as in the paper's finite-element
                 experiment), dt=1/16, 16 steps, u0=x^2(1-x)^2, 8-Gaussian f.
* ``fe_2d``      the paper's finite-element experiment (Sec. (ex-fe)):
                 [0,1]^2, constant coefficients d+-=1, alpha1=1.3,
                 alpha2=1.7, dt=0.1, f = indicator of H=[3/8,5/8]^2 (rank 1),
                 u0 = f; N=4096 per direction (the paper runs 512..65536) and
                 8 steps (the paper does not state its step count).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 180405522


def grid(n: int, left: float = 0.0, right: float = 1.0):
    """Interior grid points and spacing h = (R-L)/(N+1) (eq. (part))."""
    h = (right - left) / (n + 1)
    x = left + h * np.arange(1, n + 1, dtype=np.float64)
    return x, h


def gaussian_source(x: np.ndarray, rng: np.random.Generator, terms: int = 8):
    """sum_j a_j exp(-(x-c_j)^2 / (2 s_j^2)), a~U(-1,1), c~U(.1,.9), s~U(.01,.1)."""
    a = rng.uniform(-1.0, 1.0, terms)
    c = rng.uniform(0.1, 0.9, terms)
    s = rng.uniform(0.01, 0.1, terms)
    f = np.zeros_like(x)
    for j in range(terms):
        f += a[j] * np.exp(-((x - c[j]) ** 2) / (2.0 * s[j] ** 2))
    return f


def bump(x: np.ndarray):
    """u0(x) = x^2 (1-x)^2."""
    return x * x * (1.0 - x) ** 2


@dataclass
class Problem1D:
    """One 1D implicit-Euler problem M u^(m) = u^(m-1) + dt f (eq. (system_FD))."""
    n: int
    alpha: float
    dt: float
    steps: int
    h: float
    x: np.ndarray
    d_plus: np.ndarray
    d_minus: np.ndarray
    u0: np.ndarray
    f: np.ndarray
    name: str = ""

    @property
    def nu(self) -> float:
        return self.dt / self.h ** self.alpha


def timedep_coefficients(prob: Problem1D, t: float, amp: float = 0.25):
    """Time-dependent coefficients for a 1D problem: its d+(x), d-(x) scaled
    by 1 + amp sin(2 pi t) and 1 + amp cos(2 pi t) (both stay positive for
    amp < 1).  Returns (d_plus, d_minus) at time t."""
    return (prob.d_plus * (1.0 + amp * math.sin(2.0 * math.pi * t)),
            prob.d_minus * (1.0 + amp * math.cos(2.0 * math.pi * t)))


def plain_1d(n: int = 1024, alpha: float = 1.5, dt: float = 1.0 / 16,
             steps: int = 16) -> Problem1D:
    x, h = grid(n)
    one = np.ones(n)
    return Problem1D(n, alpha, dt, steps, h, x, one.copy(), one.copy(),
                     bump(x), np.zeros(n), name=f"plain_1d_N{n}")


def var_1d(alpha: float = 1.8, n: int = 65536, dt: float = 1.0 / 256,
           steps: int = 256, seed_offset: int = 2) -> Problem1D:
    x, h = grid(n)
    rng = np.random.default_rng(BASE_SEED + seed_offset)
    f = gaussian_source(x, rng)
    return Problem1D(n, alpha, dt, steps, h, x, 1.0 + x * x,
                     1.0 + (1.0 - x) ** 2, bump(x), f,
                     name=f"var_1d_N{n}_a{alpha}")


def batched_1d(count: int = 256, nmin: int = 2048, nmax: int = 32768,
               dt: float = 1.0 / 64, steps: int = 64,
               seed_offset: int = 3) -> list[Problem1D]:
    rng = np.random.default_rng(BASE_SEED + seed_offset)
    ns = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), count))).astype(int)
    alphas = rng.uniform(1.1, 1.9, count)
    amps = rng.uniform(0.0, 0.5, count)
    ks = rng.integers(1, 5, count)
    out = []
    for p in range(count):
        n = int(ns[p])
        x, h = grid(n)
        d = 1.0 + amps[p] * np.sin(math.pi * ks[p] * x)
        prng = np.random.default_rng(BASE_SEED + seed_offset + 1000 + p)
        out.append(Problem1D(n, float(alphas[p]), dt, steps, h, x, d.copy(), d.copy(),
                             bump(x), gaussian_source(x, prng), name=f"batch{p}_N{n}"))
    return out


@dataclass
class LowRank:
    """X = Z @ W.T with Z (nx x r), W (ny x r)."""
    Z: np.ndarray
    W: np.ndarray

    def dense(self):
        return self.Z @ self.W.T


@dataclass
class Problem2D:
    """One 2D per-step Sylvester problem A U + U B^T = U_prev + dt F (eq. (sylv-timestepping))."""
    nx: int
    ny: int
    alpha_x: float
    alpha_y: float
    dt: float
    steps: int
    hx: float
    hy: float
    x: np.ndarray
    y: np.ndarray
    dxp: np.ndarray
    dxm: np.ndarray
    dyp: np.ndarray
    dym: np.ndarray
    u0: LowRank
    f: LowRank
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def nu_x(self) -> float:
        return self.dt / self.hx ** self.alpha_x

    @property
    def nu_y(self) -> float:
        return self.dt / self.hy ** self.alpha_y


def _separable_gaussians(x, y, rng, terms, width=(0.03, 0.12), amp=(-1.0, 1.0)):
    Z = np.empty((x.size, terms))
    W = np.empty((y.size, terms))
    for j in range(terms):
        a = rng.uniform(*amp)
        cx, cy = rng.uniform(0.2, 0.8, 2)
        s = rng.uniform(*width)
        Z[:, j] = a * np.exp(-((x - cx) ** 2) / (2 * s * s))
        W[:, j] = np.exp(-((y - cy) ** 2) / (2 * s * s))
    return LowRank(Z, W)


def fd_2d(n: int = 4096, alpha_x: float = 1.3, alpha_y: float = 1.7,
          dt: float = 1.0 / 64, steps: int = 64, variable: bool = True,
          seed_offset: int = 4) -> Problem2D:
    x, hx = grid(n)
    y, hy = grid(n)
    if variable:  # eq. (coeff_es)
        g12 = math.gamma(1.2)
        dxp, dxm = g12 * (1 + x) ** alpha_x, g12 * (2 - x) ** alpha_x
        dyp, dym = g12 * (1 + y) ** alpha_y, g12 * (2 - y) ** alpha_y
    else:
        dxp = dxm = np.ones(n)
        dyp = dym = np.ones(n)
    rng = np.random.default_rng(BASE_SEED + seed_offset)
    f = _separable_gaussians(x, y, rng, 4)
    u0 = LowRank(np.zeros((n, 1)), np.zeros((n, 1)))
    return Problem2D(n, n, alpha_x, alpha_y, dt, steps, hx, hy, x, y,
                     np.asarray(dxp, float), np.asarray(dxm, float),
                     np.asarray(dyp, float), np.asarray(dym, float), u0, f,
                     name=f"fd_2d_N{n}")


def learned_2d(n: int = 2048, alpha_x: float = 1.4, alpha_y: float = 1.6,
               dt: float = 1.0 / 64, steps: int = 8, seed: int = 0) -> Problem2D:
    """One trajectory problem with a random 8-Gaussian initial condition."""
    x, hx = grid(n)
    y, hy = grid(n)
    one = np.ones(n)
    rng = np.random.default_rng(BASE_SEED + 5 + 7919 * seed)
    u0 = _separable_gaussians(x, y, rng, 8, width=(0.02, 0.1))
    f = LowRank(np.zeros((n, 1)), np.zeros((n, 1)))
    return Problem2D(n, n, alpha_x, alpha_y, dt, steps, hx, hy, x, y,
                     one, one.copy(), one.copy(), one.copy(), u0, f,
                     name=f"learned_2d_N{n}_s{seed}")


def fe_1d(n: int = 4096, alpha: float = 1.3, dt: float = 1.0 / 16,
          steps: int = 16, seed_offset: int = 6) -> Problem1D:
    """1D finite-element problem (same fields as the finite-difference ones;
    d+ = d- = 1)."""
    x, h = grid(n)
    rng = np.random.default_rng(BASE_SEED + seed_offset)
    one = np.ones(n)
    return Problem1D(n, alpha, dt, steps, h, x, one.copy(), one.copy(),
                     bump(x), gaussian_source(x, rng), name=f"fe_1d_N{n}_a{alpha}")


def fe_2d(n: int = 4096, alpha_x: float = 1.3, alpha_y: float = 1.7,
          dt: float = 0.1, steps: int = 8) -> Problem2D:
    """The finite-element experiment: f = 1 on H = [3/8, 5/8]^2, else 0;
    u(x, y, 0) = f; constant coefficients."""
    x, hx = grid(n)
    y, hy = grid(n)
    one = np.ones(n)
    ix = ((x >= 3 / 8) & (x <= 5 / 8)).astype(float)[:, None]
    iy = ((y >= 3 / 8) & (y <= 5 / 8)).astype(float)[:, None]
    f = LowRank(ix.copy(), iy.copy())
    u0 = LowRank(ix.copy(), iy.copy())
    return Problem2D(n, n, alpha_x, alpha_y, dt, steps, hx, hy, x, y,
                     one, one.copy(), one.copy(), one.copy(), u0, f,
                     name=f"fe_2d_N{n}")
