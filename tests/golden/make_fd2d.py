"""Writes the stored oracle solution of the first step of the 2D workload at
4096 x 4096 that the full-size GPU test compares against.

Calls only the oracle (Bartels-Stewart with the real Schur forms of the dense
A and B of eq. (sylv-timestepping), plus one step of iterative refinement)
and the seeded input generators; nothing
here comes from the GPU path.  The step is U^1 = X with A X + X B^T = dt F
(U^0 = 0).  X is stored as its SVD truncated where the singular values fall
below 1e-14 of the largest (Frobenius error below 1e-13 of ||X||_F, far below
the 1e-10 the test asks for): fd2d_n4096.npz holds U*s (4096 x r) and V.

Usage: python tests/golden/make_fd2d.py   (about half an hour: LAPACK's triangular
Sylvester solver runs on one core, twice)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fde2d as O2  # noqa: E402
import workloads as W  # noqa: E402

N = 4096


def main():
    p = W.fd_2d(n=N)
    t0 = time.perf_counter()
    st = O2.SylvesterStepper(p)
    t1 = time.perf_counter()
    X = st.step(np.zeros((N, N)), p.f.dense())
    t2 = time.perf_counter()
    U, sv, Vt = np.linalg.svd(X)
    r = int(np.sum(sv > 1e-14 * sv[0]))
    tail = float(np.sqrt(np.sum(sv[r:] ** 2)) / np.linalg.norm(sv))
    path = os.path.join(HERE, f"fd2d_n{N}.npz")
    np.savez(path, Z=U[:, :r] * sv[:r], W=Vt[:r].T.copy(), n=np.array(N), rank=np.array(r),
             truncation=np.array(tail))
    print(f"Schur forms {t1 - t0:.1f} s, step {t2 - t1:.1f} s; rank {r}, relative truncation {tail:.1e}; "
          f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
