"""ctypes binding of the HIP library ``libhodlr_fde.so`` (C ABI in include/hodlr_fde.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  torch supplies device memory (``data_ptr()``) and the stream.
The binding fails loudly if the library was not built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhodlr_fde.so")

HODLR_OK, HODLR_EINVAL, HODLR_ENOMEM, HODLR_EHIP, HODLR_EWORKSPACE, HODLR_ESTATE = 0, -1, -2, -3, -4, -5
HODLR_ESINGULAR, HODLR_ENOCONV, HODLR_ERANK = 1, 2, 3
FP64, MIXED_FP32, MIXED_BF16 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": MIXED_FP32, "bf16": MIXED_BF16}

# every exported symbol of include/hodlr_fde.h
EXPORTS = [
    "hodlr_ctx_create", "hodlr_ctx_destroy", "hodlr_last_arg", "hodlr_status_string",
    "hodlr_default_opts", "hodlr_build", "hodlr_destroy", "hodlr_get_info", "hodlr_matvec",
    "hodlr_toeplitz_matvec", "hodlr_factor", "hodlr_solve", "hodlr_time_steps",
    "fde2d_plan_create", "fde2d_plan_destroy", "fde2d_plan_shifts", "fde2d_sylvester_step",
    "hodlr_ctx_set_timing", "hodlr_ctx_timing_count", "hodlr_ctx_timing_entry", "hodlr_ctx_timing_reset",
    "fde2d_sylvester_step_guess", "fde2d_field_from_lr", "fde2d_compress_field", "hodlr_autotune",
    "hodlr_set_tuning", "hodlr_update_coefficients",
    "fde_net_param_count", "fde_net_create", "fde_net_destroy", "fde_net_set_params", "fde_net_get_params",
    "fde_net_get_grads", "fde_net_forward", "fde_net_train_step", "hodlr_toeplitz_matvec_noalloc",
    "hodlr_workspace_size", "hodlr_build_ws", "fde2d_plan_workspace_size", "fde2d_plan_create_ws",
    "fde2d_plan_counters", "hodlr_get_weights", "fde2d_sylvester_step_ek", "fde2d_ek_workspace_size",
    "fde2d_ek_attach_workspace",
]


FDE_FD, FDE_FE = 0, 1        # fde_discretization


class FdeOperator(C.Structure):
    _fields_ = [("n", C.c_int64), ("alpha", C.c_double), ("dt", C.c_double), ("dx", C.c_double),
                ("shift", C.c_double), ("d_plus", C.c_void_p), ("d_minus", C.c_void_p),
                ("discretization", C.c_int)]


def _fde_operator(o, default_shift):
    """fde_operator from an operator dict (see operator_dict)."""
    return FdeOperator(int(o["n"]), float(o["alpha"]), float(o["dt"]), float(o["dx"]),
                       float(o.get("shift", default_shift)), C.c_void_p(o["d_plus"].data_ptr()),
                       C.c_void_p(o["d_minus"].data_ptr()), int(o.get("discretization", FDE_FD)))


class HodlrOpts(C.Structure):
    _fields_ = [("leaf", C.c_int), ("tol", C.c_double), ("prec", C.c_int), ("max_rank", C.c_int),
                ("refine_max", C.c_int), ("rtol", C.c_double), ("gmres_m", C.c_int)]


class HodlrInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("refine_iters", C.c_int), ("rel_residual", C.c_double),
                ("max_rank", C.c_int), ("leaf", C.c_int), ("row", C.c_int),
                ("used_fallback", C.c_int), ("rel_correction", C.c_double), ("backward_error", C.c_double),
                ("guess_residual", C.c_double)]


class HodlrMatInfo(C.Structure):
    _fields_ = [("batch", C.c_int), ("leaf", C.c_int), ("max_levels", C.c_int),
                ("total_n", C.c_int64), ("max_rank_A", C.c_int), ("max_rank_factors", C.c_int),
                ("bytes_factors", C.c_size_t), ("bytes_device", C.c_size_t),
                ("factor_flops", C.c_double), ("core_flops", C.c_double), ("gram_flops", C.c_double),
                ("leaf_flops", C.c_double), ("node_rec_flops", C.c_double), ("node_pend_flops", C.c_double),
                ("sp_expand_flops", C.c_double), ("sp_project_flops", C.c_double)]


class HodlrTuning(C.Structure):
    _fields_ = [("core_threads", C.c_int), ("leaf_threads", C.c_int), ("gram_rows", C.c_int),
                ("fuse_rows", C.c_int), ("factor_ms", C.c_double)]


class LrMatrix(C.Structure):
    _fields_ = [("rows", C.c_int64), ("rank", C.c_int), ("capacity", C.c_int),
                ("ldz", C.c_int64), ("ldw", C.c_int64), ("Z", C.c_void_p), ("W", C.c_void_p)]


class Fde2dOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_shifts", C.c_int), ("max_rank", C.c_int)]


_lib = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
        L.hodlr_ctx_create.argtypes = [C.POINTER(vp), vp]
        L.hodlr_ctx_destroy.argtypes = [vp]
        L.hodlr_ctx_destroy.restype = None
        L.hodlr_last_arg.argtypes = [vp]
        L.hodlr_status_string.argtypes = [i32]
        L.hodlr_status_string.restype = C.c_char_p
        L.hodlr_default_opts.argtypes = [C.POINTER(HodlrOpts)]
        L.hodlr_build.argtypes = [vp, C.POINTER(FdeOperator), i32, C.POINTER(HodlrOpts), C.POINTER(vp)]
        L.hodlr_workspace_size.argtypes = [C.POINTER(FdeOperator), i32, C.POINTER(HodlrOpts),
                                           C.POINTER(C.c_size_t)]
        L.hodlr_build_ws.argtypes = [vp, C.POINTER(FdeOperator), i32, C.POINTER(HodlrOpts), vp, C.c_size_t,
                                     C.POINTER(vp)]
        L.hodlr_destroy.argtypes = [vp]
        L.hodlr_destroy.restype = None
        L.hodlr_get_info.argtypes = [vp, C.POINTER(HodlrMatInfo)]
        L.hodlr_matvec.argtypes = [vp, vp, vp, vp, i32, i64]
        L.hodlr_toeplitz_matvec.argtypes = [vp, vp, vp, vp, i32, i64]
        L.hodlr_toeplitz_matvec_noalloc.argtypes = [vp, vp, vp, vp, i32, i64]
        L.hodlr_factor.argtypes = [vp, vp, C.POINTER(HodlrInfo)]
        L.hodlr_solve.argtypes = [vp, vp, vp, i32, i64, C.POINTER(HodlrInfo)]
        L.hodlr_time_steps.argtypes = [vp, vp, vp, vp, dbl, i32, C.POINTER(HodlrInfo)]
        L.hodlr_autotune.argtypes = [vp, vp, C.POINTER(HodlrTuning)]
        L.hodlr_set_tuning.argtypes = [vp, vp, C.POINTER(HodlrTuning)]
        L.hodlr_update_coefficients.argtypes = [vp, vp, C.POINTER(FdeOperator)]
        L.hodlr_get_weights.argtypes = [vp, vp, i32, C.POINTER(dbl), i64]
        L.hodlr_ctx_set_timing.argtypes = [vp, i32]
        L.hodlr_ctx_timing_count.argtypes = [vp]
        L.hodlr_ctx_timing_entry.argtypes = [vp, i32, C.POINTER(C.c_char_p), C.POINTER(i64), C.POINTER(dbl)]
        L.hodlr_ctx_timing_reset.argtypes = [vp]
        L.hodlr_ctx_timing_reset.restype = None
        if hasattr(L, "fde2d_plan_create"):
            L.fde2d_plan_create.argtypes = [vp, C.POINTER(FdeOperator), C.POINTER(FdeOperator),
                                            C.POINTER(HodlrOpts), C.POINTER(Fde2dOpts), C.POINTER(vp)]
            L.fde2d_plan_workspace_size.argtypes = [vp, C.POINTER(FdeOperator), C.POINTER(FdeOperator),
                                                    C.POINTER(HodlrOpts), C.POINTER(Fde2dOpts),
                                                    C.POINTER(C.c_size_t)]
            L.fde2d_plan_create_ws.argtypes = [vp, C.POINTER(FdeOperator), C.POINTER(FdeOperator),
                                               C.POINTER(HodlrOpts), C.POINTER(Fde2dOpts), vp, C.c_size_t,
                                               C.POINTER(vp)]
            L.fde2d_plan_counters.argtypes = [vp, C.POINTER(C.c_double), i32, i32]
            L.fde2d_plan_destroy.argtypes = [vp]
            L.fde2d_plan_destroy.restype = None
            L.fde2d_plan_shifts.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double), i32]
            L.fde2d_sylvester_step.argtypes = [vp, vp, C.POINTER(LrMatrix), C.POINTER(LrMatrix), dbl,
                                               C.POINTER(LrMatrix), C.POINTER(HodlrInfo)]
            L.fde2d_sylvester_step_ek.argtypes = [vp, vp, C.POINTER(LrMatrix), C.POINTER(LrMatrix), dbl,
                                                  C.POINTER(LrMatrix), C.POINTER(HodlrInfo)]
            L.fde2d_ek_workspace_size.argtypes = [vp, vp, C.POINTER(C.c_size_t)]
            L.fde2d_ek_attach_workspace.argtypes = [vp, vp, vp, C.c_size_t]
            L.fde2d_sylvester_step_guess.argtypes = [vp, vp, C.POINTER(LrMatrix), C.POINTER(LrMatrix), dbl,
                                                     C.POINTER(LrMatrix), C.POINTER(LrMatrix), C.POINTER(HodlrInfo)]
            L.fde2d_field_from_lr.argtypes = [vp, vp, C.POINTER(LrMatrix), vp]
            L.fde2d_compress_field.argtypes = [vp, vp, vp, dbl, C.c_uint64, C.POINTER(LrMatrix)]
        if hasattr(L, "fde_net_create"):
            L.fde_net_param_count.argtypes = []
            L.fde_net_create.argtypes = [vp, i32, i64, C.POINTER(vp)]
            L.fde_net_destroy.argtypes = [vp]
            L.fde_net_destroy.restype = None
            fp = C.POINTER(C.c_float)
            L.fde_net_set_params.argtypes = [vp, vp, fp, i32]
            L.fde_net_get_params.argtypes = [vp, vp, fp, i32]
            L.fde_net_get_grads.argtypes = [vp, vp, fp, i32]
            L.fde_net_forward.argtypes = [vp, vp, vp, i32, i32, i32, vp]
            L.fde_net_train_step.argtypes = [vp, vp, vp, vp, i32, i32, i32, i32, C.c_float, i32,
                                             C.POINTER(dbl)]
        _lib = L
    return _lib


class HodlrError(RuntimeError):
    def __init__(self, status, where, ctx=None):
        msg = lib().hodlr_status_string(status).decode()
        arg = lib().hodlr_last_arg(ctx) if (ctx and status == HODLR_EINVAL) else 0
        super().__init__(f"{where}: {msg} (status {status}{', argument %d' % arg if arg else ''})")
        self.status = status


def check(status, where, ctx=None, ok=(HODLR_OK,)):
    if status not in ok:
        raise HodlrError(status, where, ctx)
    return status


def _stream_handle(torch_stream=None):
    import torch
    s = torch_stream if torch_stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Context:
    """A library context bound to one HIP stream (torch's current stream by default)."""

    def __init__(self, stream=None):
        self.h = C.c_void_p()
        check(lib().hodlr_ctx_create(C.byref(self.h), _stream_handle(stream)), "hodlr_ctx_create")

    def set_timing(self, enable: bool):
        """Bracket every kernel launched through this context with HIP events."""
        check(lib().hodlr_ctx_set_timing(self.h, int(bool(enable))), "hodlr_ctx_set_timing")

    def timing(self) -> dict:
        """{kernel launch expression: (launches, total_ms)} accumulated so far."""
        out = {}
        for i in range(lib().hodlr_ctx_timing_count(self.h)):
            name, n, ms = C.c_char_p(), C.c_int64(), C.c_double()
            check(lib().hodlr_ctx_timing_entry(self.h, i, C.byref(name), C.byref(n), C.byref(ms)),
                  "hodlr_ctx_timing_entry")
            out[name.value.decode()] = (n.value, ms.value)
        return out

    def reset_timing(self):
        lib().hodlr_ctx_timing_reset(self.h)

    def close(self):
        if self.h:
            lib().hodlr_ctx_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def default_opts(**kw) -> HodlrOpts:
    o = HodlrOpts()
    lib().hodlr_default_opts(C.byref(o))
    for k, v in kw.items():
        if k == "prec" and isinstance(v, str):
            v = PRECISIONS[v]
        setattr(o, k, v)
    return o


class HodlrMatrix:
    """A batch of HODLR-compressed operators M = s I + nu (D+ T + D- T^T)."""

    @staticmethod
    def _op_array(ops):
        arr = (FdeOperator * len(ops))()
        for i, o in enumerate(ops):
            arr[i] = _fde_operator(o, 1.0)
        return arr

    def __init__(self, ctx: Context, ops, opts: HodlrOpts, workspace: bool = True):
        """ops: list of dicts n, alpha, dt, dx, shift, d_plus, d_minus (torch CUDA float64).
        workspace=True: torch allocates the matrix's device memory (hodlr_workspace_size bytes)
        and the library builds into it (hodlr_build_ws); False: the library allocates
        (hodlr_build)."""
        self.ctx = ctx
        arr = self._op_array(ops)
        self.h = C.c_void_p()
        self.ws = None
        self.opts = opts
        self.sizes = [int(o["n"]) for o in ops]
        self.total_n = sum(self.sizes)
        if workspace:
            import torch
            need = C.c_size_t()
            check(lib().hodlr_workspace_size(arr, len(ops), C.byref(opts), C.byref(need)), "hodlr_workspace_size")
            self.ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
            if os.environ.get("HODLR_POISON") == "1":
                self.ws.fill_(0xFF)    # NaN bytes: a read of memory no kernel wrote shows in the results
            check(lib().hodlr_build_ws(ctx.h, arr, len(ops), C.byref(opts), C.c_void_p(self.ws.data_ptr()),
                                       need.value, C.byref(self.h)), "hodlr_build_ws", ctx.h)
        else:
            check(lib().hodlr_build(ctx.h, arr, len(ops), C.byref(opts), C.byref(self.h)), "hodlr_build", ctx.h)

    def update_coefficients(self, ops):
        """New d+/d- samples (same n, alpha, dt, dx, shift): rebuild the
        compressed operator in place; factor again before solving."""
        if len(ops) != len(self.sizes):
            raise ValueError("one operator per problem of the batch")
        check(lib().hodlr_update_coefficients(self.ctx.h, self.h, self._op_array(ops)),
              "hodlr_update_coefficients", self.ctx.h)

    def weights(self, item: int, count: int):
        """The generator g_0..g_{count-1} the library computed for problem `item` (numpy)."""
        import numpy as np
        out = np.zeros(int(count))
        check(lib().hodlr_get_weights(self.ctx.h, self.h, int(item),
                                      out.ctypes.data_as(C.POINTER(C.c_double)), int(count)),
              "hodlr_get_weights", self.ctx.h)
        return out

    def info(self) -> HodlrMatInfo:
        i = HodlrMatInfo()
        check(lib().hodlr_get_info(self.h, C.byref(i)), "hodlr_get_info")
        return i

    def factor(self, allow=(HODLR_OK,)) -> HodlrInfo:
        info = HodlrInfo()
        check(lib().hodlr_factor(self.ctx.h, self.h, C.byref(info)), "hodlr_factor", self.ctx.h, allow)
        return info

    def autotune(self) -> "HodlrTuning":
        """Pick the factorisation's launch shapes by timing them on this matrix
        (also used for later matrices of the same shape); factor afterwards."""
        t = HodlrTuning()
        check(lib().hodlr_autotune(self.ctx.h, self.h, C.byref(t)), "hodlr_autotune", self.ctx.h)
        return t

    def set_tuning(self, core_threads=256, leaf_threads=512, gram_rows=256, fuse_rows=256):
        """Fix the factorisation's launch shapes (see hodlr_set_tuning)."""
        t = HodlrTuning(core_threads, leaf_threads, gram_rows, fuse_rows, 0.0)
        check(lib().hodlr_set_tuning(self.ctx.h, self.h, C.byref(t)), "hodlr_set_tuning", self.ctx.h)

    def matvec(self, x, y, nrhs=1, ld=None):
        ld = self.total_n if ld is None else ld
        check(lib().hodlr_matvec(self.ctx.h, self.h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                 nrhs, ld), "hodlr_matvec", self.ctx.h)

    def toeplitz_matvec(self, x, y, nrhs=1, ld=None):
        ld = self.total_n if ld is None else ld
        check(lib().hodlr_toeplitz_matvec(self.ctx.h, self.h, C.c_void_p(x.data_ptr()),
                                          C.c_void_p(y.data_ptr()), nrhs, ld),
              "hodlr_toeplitz_matvec", self.ctx.h)

    def toeplitz_matvec_noalloc(self, x, y, nrhs=1, ld=None):
        ld = self.total_n if ld is None else ld
        check(lib().hodlr_toeplitz_matvec_noalloc(self.ctx.h, self.h, C.c_void_p(x.data_ptr()),
                                                  C.c_void_p(y.data_ptr()), nrhs, ld),
              "hodlr_toeplitz_matvec_noalloc", self.ctx.h)

    def solve(self, x, nrhs=1, ld=None, allow=(HODLR_OK,)) -> HodlrInfo:
        ld = self.total_n if ld is None else ld
        info = HodlrInfo()
        check(lib().hodlr_solve(self.ctx.h, self.h, C.c_void_p(x.data_ptr()), nrhs, ld, C.byref(info)),
              "hodlr_solve", self.ctx.h, allow)
        return info

    def time_steps(self, u, f=None, fscale=0.0, steps=1, allow=(HODLR_OK,)) -> HodlrInfo:
        info = HodlrInfo()
        fp = C.c_void_p(f.data_ptr()) if f is not None else C.c_void_p()
        check(lib().hodlr_time_steps(self.ctx.h, self.h, C.c_void_p(u.data_ptr()), fp, float(fscale),
                                     int(steps), C.byref(info)), "hodlr_time_steps", self.ctx.h, allow)
        return info

    def close(self):
        if self.h:
            lib().hodlr_destroy(self.h)     # waits for the device: the workspace is free afterwards
            self.h = C.c_void_p()
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def operator_dict(n, alpha, dt, dx, d_plus, d_minus, shift=1.0, discretization=FDE_FD):
    """One operator: FDE_FD (Grunwald-Letnikov differences) or FDE_FE (P1 finite elements)."""
    return dict(n=n, alpha=alpha, dt=dt, dx=dx, d_plus=d_plus, d_minus=d_minus, shift=shift,
                discretization=discretization)


class Fde2dPlan:
    """Shifted HODLR factor sets for A X + X B^T = C (eq. (sylv-timestepping))."""

    def __init__(self, ctx: Context, opx: dict, opy: dict, hopts: HodlrOpts, tol=1e-10, max_shifts=64,
                 max_rank=32, workspace: bool = True):
        """workspace=True: torch allocates the plan's device memory (fde2d_plan_workspace_size bytes)
        and the library builds the plan into it (fde2d_plan_create_ws)."""
        self.ctx = ctx
        self.ws = None
        self.nx, self.ny = int(opx["n"]), int(opy["n"])
        ox = _fde_operator(opx, 0.5)
        oy = _fde_operator(opy, 0.5)
        self.opts = Fde2dOpts(float(tol), int(max_shifts), int(max_rank))
        self.h = C.c_void_p()
        if workspace:
            import torch
            need = C.c_size_t()
            check(lib().fde2d_plan_workspace_size(ctx.h, C.byref(ox), C.byref(oy), C.byref(hopts),
                                                  C.byref(self.opts), C.byref(need)),
                  "fde2d_plan_workspace_size", ctx.h)
            self.ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
            check(lib().fde2d_plan_create_ws(ctx.h, C.byref(ox), C.byref(oy), C.byref(hopts), C.byref(self.opts),
                                             C.c_void_p(self.ws.data_ptr()), need.value, C.byref(self.h)),
                  "fde2d_plan_create_ws", ctx.h)
        else:
            check(lib().fde2d_plan_create(ctx.h, C.byref(ox), C.byref(oy), C.byref(hopts), C.byref(self.opts),
                                          C.byref(self.h)), "fde2d_plan_create", ctx.h)

    def counters(self, reset=False):
        """Work counters (fde2d_plan_counters): dict of core_flops, dense_flops,
        solve_bytes (one column, all shifted operators), shifts, rank, ek_shifts
        (the extended Krylov solver's projected shift pairs), ek_gemm_flops."""
        v = (C.c_double * 7)()
        check(lib().fde2d_plan_counters(self.h, v, 7, 1 if reset else 0), "fde2d_plan_counters")
        return dict(core_flops=v[0], dense_flops=v[1], solve_bytes=v[2], shifts=int(v[3]), rank=int(v[4]),
                    ek_shifts=int(v[5]), ek_gemm_flops=v[6])

    def shifts(self):
        n = lib().fde2d_plan_shifts(self.h, None, None, 0)
        p = (C.c_double * n)()
        q = (C.c_double * n)()
        lib().fde2d_plan_shifts(self.h, p, q, n)
        return list(p), list(q)

    def _lr(self, zw, cap=None, rank=None):
        Z, W = zw
        r = (Z.shape[0] if Z is not None else 0) if rank is None else rank
        return LrMatrix(self.nx, r if cap is None else 0, cap or r, self.nx, self.ny,
                        C.c_void_p(Z.data_ptr() if Z is not None and Z.numel() else 0),
                        C.c_void_p(W.data_ptr() if W is not None and W.numel() else 0))

    def step(self, Um, F, dt, out, allow=(HODLR_OK,), guess=None, guess_rank=None, ek=False):
        """Um, F, out, guess: (Z, W) pairs of column-major torch CUDA float64
        tensors stored as (rank, n) row-major (column j = row j); out gives the
        capacity.  guess: optional first guess of the solution (its first
        guess_rank columns).  ek: solve by extended Krylov
        (fde2d_sylvester_step_ek) instead of fADI sweeps."""
        a, f, o = self._lr(Um), self._lr(F), self._lr(out, cap=out[0].shape[0])
        info = HodlrInfo()
        if ek:
            if guess is not None:
                raise ValueError("the extended Krylov step takes no first guess")
            if self.ws is not None and getattr(self, "ek_ws", None) is None:
                # a workspace plan: the solver's arrays in torch-allocated memory too
                import torch
                need = C.c_size_t()
                check(lib().fde2d_ek_workspace_size(self.ctx.h, self.h, C.byref(need)), "fde2d_ek_workspace_size",
                      self.ctx.h)
                self.ek_ws = torch.empty(need.value, dtype=torch.uint8, device="cuda")
                check(lib().fde2d_ek_attach_workspace(self.ctx.h, self.h, C.c_void_p(self.ek_ws.data_ptr()),
                                                      need.value), "fde2d_ek_attach_workspace", self.ctx.h)
            check(lib().fde2d_sylvester_step_ek(self.ctx.h, self.h, C.byref(a), C.byref(f), float(dt), C.byref(o),
                                                C.byref(info)), "fde2d_sylvester_step_ek", self.ctx.h, allow)
        elif guess is None:
            check(lib().fde2d_sylvester_step(self.ctx.h, self.h, C.byref(a), C.byref(f), float(dt), C.byref(o),
                                             C.byref(info)), "fde2d_sylvester_step", self.ctx.h, allow)
        else:
            g = self._lr(guess, rank=guess_rank)
            check(lib().fde2d_sylvester_step_guess(self.ctx.h, self.h, C.byref(a), C.byref(f), float(dt),
                                                   C.byref(g), C.byref(o), C.byref(info)),
                  "fde2d_sylvester_step_guess", self.ctx.h, allow)
        return o.rank, info

    def to_field(self, zw, out, rank=None):
        """Dense FP32 field of X = Z W^T into out, a (ny, nx) torch CUDA float32
        tensor (row j = grid line y_j)."""
        x = self._lr(zw, rank=rank)
        check(lib().fde2d_field_from_lr(self.ctx.h, self.h, C.byref(x), C.c_void_p(out.data_ptr())),
              "fde2d_field_from_lr", self.ctx.h)

    def compress_field(self, field, tol, out, seed=1):
        """Low-rank (Z, W) of a dense (ny, nx) FP32 field; out gives the capacity; returns the rank."""
        o = self._lr(out, cap=out[0].shape[0])
        check(lib().fde2d_compress_field(self.ctx.h, self.h, C.c_void_p(field.data_ptr()), float(tol), int(seed),
                                         C.byref(o)), "fde2d_compress_field", self.ctx.h)
        return o.rank

    def close(self):
        if self.h:
            lib().fde2d_plan_destroy(self.h)    # its batches' destruction waits for the device
            self.h = C.c_void_p()
        self.ws = None
        self.ek_ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ConvNet:
    """The learned warm start's network (four 3x3 convolutions, 1 -> 32 -> 32 ->
    32 -> 1, residual output u + net(u)), trained and run by the library's
    kernels.  Parameters use the layout of fde_net_set_params."""

    def __init__(self, ctx: Context, bf16=True, max_pixels=1 << 22):
        self.ctx = ctx
        self.h = C.c_void_p()
        self.count = lib().fde_net_param_count()
        check(lib().fde_net_create(ctx.h, int(bool(bf16)), int(max_pixels), C.byref(self.h)), "fde_net_create",
              ctx.h)

    @staticmethod
    def flatten(params):
        """[[w1, b1], ..., [w4, b4]] (numpy, oracle layout) -> float32 vector."""
        import numpy as np
        return np.concatenate([np.asarray(a, dtype=np.float32).ravel() for wb in params for a in wb])

    @staticmethod
    def unflatten(flat, channels=32):
        import numpy as np
        shapes = [(channels, 1, 3, 3), (channels,), (channels, channels, 3, 3), (channels,),
                  (channels, channels, 3, 3), (channels,), (1, channels, 3, 3), (1,)]
        out, off = [], 0
        for s in shapes:
            n = int(np.prod(s))
            out.append(np.asarray(flat[off:off + n], dtype=np.float64).reshape(s))
            off += n
        return [out[0:2], out[2:4], out[4:6], out[6:8]]

    def set_params(self, params):
        import numpy as np
        flat = params if isinstance(params, np.ndarray) else self.flatten(params)
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        check(lib().fde_net_set_params(self.ctx.h, self.h, flat.ctypes.data_as(C.POINTER(C.c_float)), self.count),
              "fde_net_set_params", self.ctx.h)

    def _get(self, fn, name):
        import numpy as np
        out = np.zeros(self.count, dtype=np.float32)
        check(fn(self.ctx.h, self.h, out.ctypes.data_as(C.POINTER(C.c_float)), self.count), name, self.ctx.h)
        return out

    def get_params(self):
        return self._get(lib().fde_net_get_params, "fde_net_get_params")

    def get_grads(self):
        return self._get(lib().fde_net_get_grads, "fde_net_get_grads")

    def forward(self, u, pred):
        """u, pred: (n, h, w) torch CUDA float32 tensors."""
        n, hh, ww = u.shape
        check(lib().fde_net_forward(self.ctx.h, self.h, C.c_void_p(u.data_ptr()), n, hh, ww,
                                    C.c_void_p(pred.data_ptr())), "fde_net_forward", self.ctx.h)

    def train_step(self, u, target, margin=4, lr=1e-3, update=True):
        n, hh, ww = u.shape
        loss = C.c_double()
        check(lib().fde_net_train_step(self.ctx.h, self.h, C.c_void_p(u.data_ptr()), C.c_void_p(target.data_ptr()),
                                       n, hh, ww, int(margin), float(lr), int(bool(update)), C.byref(loss)),
              "fde_net_train_step", self.ctx.h)
        return loss.value

    def close(self):
        if self.h:
            lib().fde_net_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
