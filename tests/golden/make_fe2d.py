"""Writes the stored oracle solution of the first step of the 2D
finite-element workload at 4096 x 4096 that the full-size GPU test compares
against.

Calls only the oracle (the generalized Sylvester step of eq.
(sylv-timestepping-fe) by the paper's route: mass matrices inverted,
Bartels-Stewart with the real Schur forms, one step of iterative refinement
on the generalized equation) and the seeded input generators; nothing here
comes from the GPU path.  The step is U^1 = X with
A X E_y + E_x X B^T = E_x (U^0 + dt F) E_y, U^0 = F = the indicator of
[3/8, 5/8]^2.  X is stored as its SVD truncated where the singular values
fall below 1e-14 of the largest: fe2d_n4096.npz holds U*s (4096 x r) and V.

Usage: python tests/golden/make_fe2d.py   (about half an hour: LAPACK's
triangular Sylvester solver runs on one core)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fe as OF  # noqa: E402
import workloads as W  # noqa: E402

N = 4096


def main():
    p = W.fe_2d(n=N)
    t0 = time.perf_counter()
    st = OF.FeSylvesterStepper(p)
    t1 = time.perf_counter()
    X = st.step(p.u0.dense(), p.f.dense(), refine=1)
    t2 = time.perf_counter()
    U, sv, Vt = np.linalg.svd(X)
    r = int(np.sum(sv > 1e-14 * sv[0]))
    tail = float(np.sqrt(np.sum(sv[r:] ** 2)) / np.linalg.norm(sv))
    path = os.path.join(HERE, f"fe2d_n{N}.npz")
    np.savez(path, Z=U[:, :r] * sv[:r], W=Vt[:r].T.copy(), n=np.array(N), rank=np.array(r),
             truncation=np.array(tail))
    print(f"Schur forms {t1 - t0:.1f} s, step {t2 - t1:.1f} s; rank {r}, relative truncation {tail:.1e}; "
          f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
