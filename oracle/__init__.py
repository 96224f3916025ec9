"""Plain FP64 CPU oracle for the HODLR fractional-diffusion solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute
anything in this package.  The product library (HIP kernels behind the C ABI)
never does, and this package never imports the product.  The two sides share
only ``workloads.py``, which generates seeded inputs and holds none of the
method's arithmetic.

Modules:
* ``fde1d``   Grunwald-Letnikov weights, dense M of eq. (system_FD), implicit
              Euler with dense LU + double-double refinement, manufactured
              solution, rank-structure helpers.
* ``fde2d``   dense A, B of eq. (sylv-timestepping); Kronecker brute force,
              Bartels-Stewart and symmetric eigen-solves of the per-step
              Sylvester equation.
* ``convnet`` FP64 forward/backward of the warm-start network, MSE, Adam.

Every function here is pinned by ``tests/test_oracle_*.py`` (``-m "not gpu"``)
against closed forms, textbook routines, brute force or values printed in the
paper, except where its docstring says "parity unpinned".
"""
