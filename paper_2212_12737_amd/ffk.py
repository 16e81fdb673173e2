"""Python binding of libffkrr (ctypes).

Argument marshalling only: every step runs in the HIP library.  Device memory
and streams come from PyTorch (ROCm build); tensors are passed as raw device
pointers.  The functions carry the names of the C entry points without the
``ffk_`` prefix.  A missing library raises immediately -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libffkrr.so")

FP64, FP32, BF16, BF16X3 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "bf16x3": BF16X3}
UNIFORM, LEVERAGE, PIVCHOL, SCORES = 0, 1, 2, 3
STRATEGIES = {"uniform": UNIFORM, "leverage": LEVERAGE, "pivchol": PIVCHOL, "scores": SCORES}
OK, NOT_CONVERGED, WARN_RANK_DROPPED = 0, 1, 2

_lib = None


class FfkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("ffkrr error %d: %s" % (status, msg))
        self.status = status


class PcgOpts(ctypes.Structure):
    _fields_ = [("lam", ctypes.c_double), ("tol", ctypes.c_double), ("max_iter", ctypes.c_int64),
                ("prec", ctypes.c_int32), ("refresh_every", ctypes.c_int32), ("escalate", ctypes.c_int32),
                ("flexible", ctypes.c_int32), ("timing", ctypes.c_int32), ("switch_below", ctypes.c_double),
                ("progress_every", ctypes.c_int32), ("switch_from", ctypes.c_int32),
                ("gap_escalate", ctypes.c_double), ("resume", ctypes.c_int32),
                ("direction", ctypes.c_void_p)]


class PcgReport(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("n_refresh", ctypes.c_int64), ("n_escalations", ctypes.c_int64),
                ("rel_res_true", ctypes.c_double), ("rel_res_updated", ctypes.c_double),
                ("final_prec", ctypes.c_int32), ("status", ctypes.c_int32),
                ("switch_iter", ctypes.c_int64), ("esc_iter", ctypes.c_int64 * 3),
                ("t_mvm_ms", ctypes.c_double), ("t_prec_ms", ctypes.c_double), ("t_vec_ms", ctypes.c_double),
                ("t_refresh_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double),
                ("hist_host", ctypes.POINTER(ctypes.c_double)), ("hist_cap", ctypes.c_int64),
                ("hist_len", ctypes.c_int64)]


P = ctypes.c_void_p
I64, I32, U64, DBL, FLT = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double, ctypes.c_float
PP = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "ffk_create": (I32, [PP, I32]),
    "ffk_destroy": (None, [P]),
    "ffk_last_error": (ctypes.c_char_p, [P]),
    "ffk_version": (ctypes.c_char_p, []),
    "ffk_descriptor_build": (I32, [P, P, I64, I32, DBL, PP, P]),
    "ffk_system_free": (None, [P]),
    "ffk_system_info": (I32, [P, ctypes.POINTER(I64), ctypes.POINTER(I32), ctypes.POINTER(I64), ctypes.POINTER(I64)]),
    "ffk_descriptor_export": (I32, [P, P, P, P]),
    "ffk_kernel_mvm": (I32, [P, P, P, P, DBL, I32, P]),
    "ffk_kernel_mvm_noalloc": (I32, [P, P, P, P, DBL, I32, P]),
    "ffk_kernel_mvm_phases": (I32, [P, P, P, P, DBL, I32, I32, ctypes.POINTER(DBL), P]),
    "ffk_clock_enable": (I32, [P, I32]),
    "ffk_clock_read": (I32, [P, I32, ctypes.POINTER(DBL), ctypes.POINTER(I64)]),
    "ffk_kernel_predict": (I32, [P, P, P, P, P, P]),
    "ffk_kernel_columns": (I32, [P, P, P, I64, P, P]),
    "ffk_kernel_diag": (I32, [P, P, P, P]),
    "ffk_nystrom_select": (I32, [P, P, I32, I64, DBL, U64, I64, P, P, ctypes.POINTER(I64), P, P]),
    "ffk_precond_build": (I32, [P, P, P, I64, DBL, I32, PP, P]),
    "ffk_precond_build_ex": (I32, [P, P, P, I64, DBL, I32, I32, PP, P]),
    "ffk_precond_free": (None, [P]),
    "ffk_precond_info": (I32, [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64)]),
    "ffk_precond_apply": (I32, [P, P, P, P, P]),
    "ffk_precond_export": (I32, [P, P, P, P]),
    "ffk_pcg_solve": (I32, [P, P, P, P, P, ctypes.POINTER(PcgOpts), ctypes.POINTER(PcgReport), P]),
    "ffk_exact_rls": (I32, [P, P, DBL, P, P]),
    "ffk_mlp_create": (I32, [P, I32, I32, U64, PP]),
    "ffk_mlp_free": (None, [P]),
    "ffk_mlp_num_params": (I64, [I32, I32]),
    "ffk_mlp_set_params": (I32, [P, P, P, P]),
    "ffk_mlp_get_params": (I32, [P, P, P, P]),
    "ffk_mlp_set_norm": (I32, [P, P, P, P, P]),
    "ffk_mlp_forward": (I32, [P, P, P, I64, P, I32, P]),
    "ffk_mlp_grad": (I32, [P, P, P, P, I64, P, P, P]),
    "ffk_mlp_adam_step": (I32, [P, P, P, FLT, P]),
    "ffk_mlp_scores": (I32, [P, P, P, P, P]),
    "ffk_block_log_scores": (I32, [P, P, I64, I32, P, P]),
    "ffk_mlp_prepare_inputs": (I32, [P, P, P, P, I32, P]),
    "ffk_mlp_fit_norm": (I32, [P, P, P, I64, P]),
    "ffk_rule_of_thumb": (I64, [I64, DBL, DBL]),
    "ffk_system_set_symmetries": (I32, [P, P, P, I32, P]),
    "ffk_rot_fit": (I32, [P, P, I32, I64, P, P]),
    "ffk_rule_of_thumb_calibrated": (I64, [I64, DBL, DBL, DBL, DBL, DBL]),
}


def lib():
    """Load libffkrr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libffkrr.so is not built: run `python -m paper_2212_12737_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS)


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor | None, dtype=None):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError("expected %s, got %s" % (dtype, t.dtype))
    if not t.is_contiguous() and not (t.dim() == 2 and t.t().is_contiguous()):
        raise ValueError("expected a densely packed tensor")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        st = lib().ffk_create(ctypes.byref(h), device)
        if st != OK:
            raise FfkError(st, "ffk_create failed for device %d" % device)
        self.h = h
        self.device = device
        self.torch_device = torch.device("cuda", device)

    def check(self, st: int, what: str) -> int:
        if st < 0:
            raise FfkError(st, "%s: %s" % (what, lib().ffk_last_error(self.h).decode()))
        return st

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ffk_destroy(self.h)
            self.h = None


def create(device: int = 0) -> Context:
    return Context(device)


def version() -> str:
    return lib().ffk_version().decode()


class System:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h
        N, M, D, n = I64(), I32(), I64(), I64()
        lib().ffk_system_info(h, ctypes.byref(N), ctypes.byref(M), ctypes.byref(D), ctypes.byref(n))
        self.N, self.M, self.D, self.n = N.value, M.value, D.value, n.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ffk_system_free(self.h)
            self.h = None


def descriptor_build(ctx: Context, R: torch.Tensor, sigma: float, stream=None) -> System:
    R = R.to(device=ctx.torch_device, dtype=torch.float64).contiguous()
    N, M, _ = R.shape
    h = ctypes.c_void_p()
    ctx.check(lib().ffk_descriptor_build(ctx.h, _ptr(R), N, M, sigma, ctypes.byref(h), _stream(stream)),
              "descriptor_build")
    return System(ctx, h)


def descriptor_export(ctx: Context, sys: System, stream=None) -> torch.Tensor:
    X = torch.empty((sys.N, sys.D), dtype=torch.float64, device=ctx.torch_device)
    ctx.check(lib().ffk_descriptor_export(ctx.h, sys.h, _ptr(X), _stream(stream)), "descriptor_export")
    return X


def kernel_mvm(ctx: Context, sys: System, v: torch.Tensor, y: torch.Tensor | None = None, shift: float = 0.0,
               prec: int = FP64, stream=None) -> torch.Tensor:
    if y is None:
        y = torch.empty(sys.n, dtype=torch.float64, device=ctx.torch_device)
    ctx.check(lib().ffk_kernel_mvm(ctx.h, sys.h, _ptr(v, torch.float64), _ptr(y, torch.float64), shift, prec,
                                   _stream(stream)), "kernel_mvm")
    return y


def kernel_mvm_noalloc(ctx: Context, sys: System, v: torch.Tensor, y: torch.Tensor, shift: float = 0.0,
                       prec: int = FP64, stream=None) -> torch.Tensor:
    """ffk_kernel_mvm_noalloc: the product with the library's fixed scratch as workspace (y must be given)."""
    ctx.check(lib().ffk_kernel_mvm_noalloc(ctx.h, sys.h, _ptr(v, torch.float64), _ptr(y, torch.float64), shift,
                                           prec, _stream(stream)), "kernel_mvm_noalloc")
    return y


MVM_PHASES = ("jv", "colsum", "gemm1", "gemm2", "jtg")


def kernel_mvm_phases(ctx: Context, sys: System, v: torch.Tensor, prec: int = FP64, iters: int = 10,
                      shift: float = 0.0, stream=None) -> dict:
    y = torch.empty(sys.n, dtype=torch.float64, device=ctx.torch_device)
    ms = (DBL * 5)()
    ctx.check(lib().ffk_kernel_mvm_phases(ctx.h, sys.h, _ptr(v, torch.float64), _ptr(y), shift, prec, iters, ms,
                                          _stream(stream)), "kernel_mvm_phases")
    return dict(zip(MVM_PHASES, list(ms)))


CLOCKS = ("jv", "colsum", "gemm1", "gemm2", "gemm2_reduce", "jtg", "gemv_t", "gemv_n", "core", "fused")


def clock_enable(ctx: Context, stride: int = 1) -> None:
    """Zero the kernel clocks and time every stride-th launch (0 stops recording)."""
    ctx.check(lib().ffk_clock_enable(ctx.h, int(stride)), "clock_enable")


def clock_read(ctx: Context) -> dict:
    """{kernel: (total_ms, timed launches)} for every clock; synchronizes the device."""
    out = {}
    for i, name in enumerate(CLOCKS):
        ms, cnt = DBL(0.0), I64(0)
        ctx.check(lib().ffk_clock_read(ctx.h, i, ctypes.byref(ms), ctypes.byref(cnt)), "clock_read")
        out[name] = (ms.value, cnt.value)
    return out


def set_symmetries(ctx: Context, sys: System, perms, stream=None) -> None:
    """Symmetrize the kernel of sys over a group of atom permutations (S x M rows p_q)."""
    import numpy as np
    P = np.ascontiguousarray(np.asarray(perms, dtype=np.int32))
    if P.ndim != 2 or P.shape[1] != sys.M:
        raise ValueError("perms must be S x M")
    ctx.check(lib().ffk_system_set_symmetries(ctx.h, sys.h, P.ctypes.data, P.shape[0], _stream(stream)),
              "set_symmetries")


def kernel_predict(ctx: Context, train: System, test: System, alpha: torch.Tensor, stream=None) -> torch.Tensor:
    F = torch.empty(test.n, dtype=torch.float64, device=ctx.torch_device)
    ctx.check(lib().ffk_kernel_predict(ctx.h, train.h, test.h, _ptr(alpha, torch.float64), _ptr(F), _stream(stream)),
              "kernel_predict")
    return F


def kernel_columns(ctx: Context, sys: System, cols: torch.Tensor, stream=None) -> torch.Tensor:
    cols = cols.to(device=ctx.torch_device, dtype=torch.int64).contiguous()
    k = cols.numel()
    out = torch.empty((k, sys.n), dtype=torch.float64, device=ctx.torch_device)
    ctx.check(lib().ffk_kernel_columns(ctx.h, sys.h, _ptr(cols), k, _ptr(out), _stream(stream)), "kernel_columns")
    return out.t()


def kernel_diag(ctx: Context, sys: System, stream=None) -> torch.Tensor:
    d = torch.empty(sys.n, dtype=torch.float64, device=ctx.torch_device)
    ctx.check(lib().ffk_kernel_diag(ctx.h, sys.h, _ptr(d), _stream(stream)), "kernel_diag")
    return d


def nystrom_select(ctx: Context, sys: System, strategy, k: int, lam: float = 0.0, seed: int = 0, pilot: int = 0,
                   weights: torch.Tensor | None = None, return_tau: bool = False, stream=None):
    strategy = STRATEGIES[strategy] if isinstance(strategy, str) else strategy
    idx = torch.empty(k, dtype=torch.int64, device=ctx.torch_device)
    keff = I64()
    tau = torch.empty(sys.n, dtype=torch.float64, device=ctx.torch_device) if return_tau else None
    if weights is not None:
        weights = weights.to(device=ctx.torch_device, dtype=torch.float64).contiguous()
    ctx.check(lib().ffk_nystrom_select(ctx.h, sys.h, strategy, k, lam, seed & (2 ** 64 - 1), pilot, _ptr(weights),
                                       _ptr(idx), ctypes.byref(keff), _ptr(tau), _stream(stream)), "nystrom_select")
    idx = idx[:keff.value]
    return (idx, tau) if return_tau else idx


class Precond:
    def __init__(self, ctx: Context, h, status: int):
        self.ctx, self.h = ctx, h
        self.dropped = status == WARN_RANK_DROPPED
        k, keff, nb = I64(), I64(), I64()
        lib().ffk_precond_info(h, ctypes.byref(k), ctypes.byref(keff), ctypes.byref(nb))
        self.k, self.k_eff, self.bytes = k.value, keff.value, nb.value
        self.sys = None   # a matrix-free preconditioner keeps its system alive here

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ffk_precond_free(self.h)
            self.h = None


BUILD_LOWMEM, BUILD_MATRIX_FREE = 1, 2


def precond_build(ctx: Context, sys: System, idx: torch.Tensor, lam: float, store: int = FP64,
                  lowmem: bool = False, matrix_free: bool = False, stream=None) -> Precond:
    idx = idx.to(device=ctx.torch_device, dtype=torch.int64).contiguous()
    h = ctypes.c_void_p()
    flags = (BUILD_LOWMEM if lowmem else 0) | (BUILD_MATRIX_FREE if matrix_free else 0)
    st = ctx.check(lib().ffk_precond_build_ex(ctx.h, sys.h, _ptr(idx), idx.numel(), lam, store, flags,
                                              ctypes.byref(h), _stream(stream)), "precond_build")
    P = Precond(ctx, h, st)
    if matrix_free:
        P.sys = sys
    return P


def precond_apply(ctx: Context, P: Precond, r: torch.Tensor, z: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    if z is None:
        z = torch.empty_like(r)
    ctx.check(lib().ffk_precond_apply(ctx.h, P.h, _ptr(r, torch.float64), _ptr(z, torch.float64), _stream(stream)),
              "precond_apply")
    return z


def precond_export(ctx: Context, P: Precond, n: int, stream=None) -> torch.Tensor:
    L = torch.empty((P.k_eff, n), dtype=torch.float64, device=ctx.torch_device)
    ctx.check(lib().ffk_precond_export(ctx.h, P.h, _ptr(L), _stream(stream)), "precond_export")
    return L.t()


@dataclass
class Report:
    status: int
    iters: int
    n_refresh: int
    n_escalations: int
    rel_res_true: float
    rel_res_updated: float
    final_prec: int
    t_mvm_ms: float
    t_prec_ms: float
    t_vec_ms: float
    t_refresh_ms: float
    t_total_ms: float
    hist: list
    switch_iter: int = -1
    esc_iter: tuple = ()


# Mixed-precision schedule used by the benchmark and the studies: FP32
# products (MIXED_SWITCH_FROM) until the recursive residual is below
# MIXED_SWITCH_BELOW |F|, the reduced precision afterwards, and an FP64
# true-residual refresh every MIXED_REFRESH iterations (measured best on the
# M=21, N=2000 system: switch points 0.01 .. 0.95, refresh intervals 5, 10 and
# 20, FP64 or FP32 before the switch; FP32 before the switch also measured
# faster at N=10000).
MIXED_SWITCH_BELOW = 0.7
MIXED_REFRESH = 10
MIXED_SWITCH_FROM = FP32


def pcg_solve(ctx: Context, sys: System, P: Precond | None, F: torch.Tensor, lam: float, tol: float = 1e-6,
              max_iter: int = 0, prec: int = FP64, refresh_every: int = 10, escalate: bool = True,
              flexible: bool = False, timing: bool = False, hist_cap: int = 0, alpha: torch.Tensor | None = None,
              switch_below: float = 0.0, progress_every: int = 0, switch_from: int = FP64,
              gap_escalate: float = 0.0, resume: bool = False, direction: torch.Tensor | None = None,
              stream=None):
    """resume: start from the content of `alpha` (required then).  direction:
    with resume, the search direction to continue along (None: restart);
    in every case it receives the direction of the next iteration."""
    if alpha is None:
        if resume:
            raise ValueError("pcg_solve: resume needs the starting alpha")
        alpha = torch.empty(sys.n, dtype=torch.float64, device=ctx.torch_device)
    o = PcgOpts(lam, tol, max_iter, prec, refresh_every, int(escalate), int(flexible), int(timing), switch_below,
                int(progress_every), int(switch_from), float(gap_escalate), int(resume),
                _ptr(direction, torch.float64) if direction is not None else None)
    rep = PcgReport()
    hist = (ctypes.c_double * hist_cap)() if hist_cap > 0 else None
    if hist is not None:
        rep.hist_host = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        rep.hist_cap = hist_cap
    st = ctx.check(lib().ffk_pcg_solve(ctx.h, sys.h, P.h if P is not None else None, _ptr(F, torch.float64),
                                       _ptr(alpha, torch.float64), ctypes.byref(o), ctypes.byref(rep),
                                       _stream(stream)), "pcg_solve")
    r = Report(st, rep.iters, rep.n_refresh, rep.n_escalations, rep.rel_res_true, rep.rel_res_updated,
               rep.final_prec, rep.t_mvm_ms, rep.t_prec_ms, rep.t_vec_ms, rep.t_refresh_ms, rep.t_total_ms,
               list(hist[:rep.hist_len]) if hist is not None else [], rep.switch_iter, tuple(rep.esc_iter))
    return alpha, r


def exact_rls(ctx: Context, sys: System, lam: float, stream=None) -> torch.Tensor:
    tau = torch.empty(sys.n, dtype=torch.float64, device=ctx.torch_device)
    ctx.check(lib().ffk_exact_rls(ctx.h, sys.h, lam, _ptr(tau), _stream(stream)), "exact_rls")
    return tau


class Mlp:
    def __init__(self, ctx: Context, h, D: int, H: int):
        self.ctx, self.h, self.D, self.H = ctx, h, D, H
        self.nparam = lib().ffk_mlp_num_params(D, H)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ffk_mlp_free(self.h)
            self.h = None


def mlp_num_params(D: int, H: int) -> int:
    return lib().ffk_mlp_num_params(D, H)


def mlp_create(ctx: Context, D: int, H: int = 256, seed: int = 0) -> Mlp:
    h = ctypes.c_void_p()
    ctx.check(lib().ffk_mlp_create(ctx.h, D, H, seed, ctypes.byref(h)), "mlp_create")
    return Mlp(ctx, h, D, H)


def mlp_set_params(ctx: Context, net: Mlp, theta: torch.Tensor, stream=None):
    ctx.check(lib().ffk_mlp_set_params(ctx.h, net.h, _ptr(theta, torch.float32), _stream(stream)), "mlp_set_params")


def mlp_get_params(ctx: Context, net: Mlp, stream=None) -> torch.Tensor:
    t = torch.empty(net.nparam, dtype=torch.float32, device=ctx.torch_device)
    ctx.check(lib().ffk_mlp_get_params(ctx.h, net.h, _ptr(t), _stream(stream)), "mlp_get_params")
    return t


def mlp_set_norm(ctx: Context, net: Mlp, mean: torch.Tensor, inv_std: torch.Tensor, stream=None):
    mean = mean.to(device=ctx.torch_device, dtype=torch.float32).contiguous()
    inv_std = inv_std.to(device=ctx.torch_device, dtype=torch.float32).contiguous()
    ctx.check(lib().ffk_mlp_set_norm(ctx.h, net.h, _ptr(mean), _ptr(inv_std), _stream(stream)), "mlp_set_norm")


def mlp_forward(ctx: Context, net: Mlp, X: torch.Tensor, prec: int = FP32, stream=None) -> torch.Tensor:
    out = torch.empty(X.shape[0], dtype=torch.float32, device=ctx.torch_device)
    ctx.check(lib().ffk_mlp_forward(ctx.h, net.h, _ptr(X, torch.float32), X.shape[0], _ptr(out), prec,
                                    _stream(stream)), "mlp_forward")
    return out


def mlp_grad(ctx: Context, net: Mlp, X: torch.Tensor, y: torch.Tensor, stream=None):
    loss = torch.empty(1, dtype=torch.float32, device=ctx.torch_device)
    grad = torch.empty(net.nparam, dtype=torch.float32, device=ctx.torch_device)
    ctx.check(lib().ffk_mlp_grad(ctx.h, net.h, _ptr(X, torch.float32), _ptr(y, torch.float32), X.shape[0],
                                 _ptr(loss), _ptr(grad), _stream(stream)), "mlp_grad")
    return loss, grad


def mlp_adam_step(ctx: Context, net: Mlp, grad: torch.Tensor, lr: float, stream=None):
    ctx.check(lib().ffk_mlp_adam_step(ctx.h, net.h, _ptr(grad, torch.float32), lr, _stream(stream)),
              "mlp_adam_step")


def mlp_scores(ctx: Context, net: Mlp, sys: System, stream=None) -> torch.Tensor:
    s = torch.empty(sys.N, dtype=torch.float64, device=ctx.torch_device)
    ctx.check(lib().ffk_mlp_scores(ctx.h, net.h, sys.h, _ptr(s), _stream(stream)), "mlp_scores")
    return s


def block_log_scores(ctx: Context, tau: torch.Tensor, N: int, M: int, stream=None) -> torch.Tensor:
    y = torch.empty(N, dtype=torch.float32, device=ctx.torch_device)
    ctx.check(lib().ffk_block_log_scores(ctx.h, _ptr(tau, torch.float64), N, M, _ptr(y), _stream(stream)),
              "block_log_scores")
    return y


def mlp_prepare_inputs(ctx: Context, net: Mlp, sys: System, standardize: bool = True, out=None,
                       stream=None) -> torch.Tensor:
    X = out if out is not None else torch.empty((sys.N, sys.D), dtype=torch.float32, device=ctx.torch_device)
    ctx.check(lib().ffk_mlp_prepare_inputs(ctx.h, net.h, sys.h, _ptr(X, torch.float32), int(standardize),
                                           _stream(stream)), "mlp_prepare_inputs")
    return X


def mlp_fit_norm(ctx: Context, net: Mlp, X: torch.Tensor, stream=None):
    ctx.check(lib().ffk_mlp_fit_norm(ctx.h, net.h, _ptr(X, torch.float32), X.shape[0], _stream(stream)),
              "mlp_fit_norm")


def rule_of_thumb(n: int, k_min: float = 100.0, m: float = 1.0) -> int:
    return int(lib().ffk_rule_of_thumb(n, k_min, m))


def rule_of_thumb_calibrated(n: int, k_min: float, m: float, a: float, b: float, c: float) -> int:
    """argmin over k of n (k_min/k)^m (a + b k) + c k^2 (Eq. 7 with measured costs)."""
    return int(lib().ffk_rule_of_thumb_calibrated(n, k_min, m, a, b, c))


def rot_fit(k, iters, n: int) -> tuple[float, float]:
    """(k_min, m) of the power law #/n = (k_min/k)^m fitted to measured (k, #) pairs."""
    kk = (ctypes.c_int64 * len(k))(*[int(x) for x in k])
    it = (ctypes.c_int64 * len(iters))(*[int(x) for x in iters])
    kmin, m = ctypes.c_double(), ctypes.c_double()
    st = lib().ffk_rot_fit(kk, it, len(k), int(n), ctypes.byref(kmin), ctypes.byref(m))
    if st != 0:
        raise FfkError(st, "rot_fit: need >= 2 distinct k with iterations that fall with k")
    return kmin.value, m.value
