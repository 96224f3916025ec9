"""HODLR solver for space-fractional diffusion equations on MI355X (gfx950).

The compute path is the HIP library ``libhodlr_fde.so`` (C ABI declared in
``include/hodlr_fde.h``); :mod:`paper_1804_05522_amd.hodlr` is its ctypes
binding.  torch provides device memory and streams only.
"""
from .hodlr import (Context, HodlrMatrix, HodlrError, Fde2dPlan, ConvNet, default_opts, lib, operator_dict,  # noqa: F401
                    FP64, MIXED_FP32, MIXED_BF16, FDE_FD, FDE_FE, EXPORTS)
