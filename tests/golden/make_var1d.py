"""Writes the stored oracle trajectories of the 1D variable-coefficient
workload that the full-size GPU parity tests compare against.

Calls only the oracle (dense LU of the implicit-Euler matrix of eq.
(system_FD), steps refined with the double-double residual) and the seeded
input generators; nothing here comes from the GPU path.

  var1d_n16384.npz  N = 16384, alpha in {1.2, 1.8}, dt = 1/256: u^(m) at
                    m = 1, 2, 4, ..., 256 (the whole 256-step trajectory,
                    sampled at powers of two)
  var1d_n65536.npz  N = 65536 (the benchmark's size), alpha in {1.2, 1.8},
                    dt = 1/256: u^(m) at m = 1, 2, 3, 4 (dense LU of a 34 GB
                    matrix, built in place; about 10 minutes per alpha on 8
                    cores)

Usage: python tests/golden/make_var1d.py [16384|65536 ...]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fde1d as O  # noqa: E402
import workloads as W  # noqa: E402

STORED = {16384: [1, 2, 4, 8, 16, 32, 64, 128, 256], 65536: [1, 2, 3, 4]}
ALPHAS = (1.2, 1.8)


def trajectory(alpha: float, n: int, keep: list[int]) -> np.ndarray:
    p = W.var_1d(alpha, n=n)
    t0 = time.perf_counter()
    S = O.DenseSolver(p.alpha, p.n, p.nu, p.d_plus, p.d_minus, lean=True)
    print(f"  N={n} alpha={alpha}: LU {time.perf_counter() - t0:.1f} s", flush=True)
    u = p.u0.copy()
    out = []
    for m in range(1, max(keep) + 1):
        u = S.solve(u + p.dt * p.f)
        if m in keep:
            out.append(u.copy())
    del S
    return np.stack(out)


def main(sizes):
    for n in sizes:
        keep = STORED[n]
        data = {"steps": np.array(keep), "alphas": np.array(ALPHAS), "n": np.array(n)}
        for a in ALPHAS:
            t0 = time.perf_counter()
            data[f"u_a{a}"] = trajectory(a, n, keep)
            print(f"  N={n} alpha={a}: {time.perf_counter() - t0:.1f} s", flush=True)
        path = os.path.join(HERE, f"var1d_n{n}.npz")
        np.savez(path, **data)
        print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or sorted(STORED))
