"""ctypes binding of libtgv.so (C-ABI declared in include/tgv.h).

Argument marshalling only: every computation runs in the HIP kernels behind
the C-ABI.  Functions keep the C names; arrays are torch tensors on the GPU
(shape (5, nz, ny, nx) for state-like arrays, contiguous), streams default to
torch's current stream.  A missing library raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libtgv.so")

NS_F64, NS_F32, NS_F16, NS_BF16 = 0, 1, 2, 3
_TORCH_OF = {NS_F64: torch.float64, NS_F32: torch.float32, NS_F16: torch.float16, NS_BF16: torch.bfloat16}
_CODE_OF = {v: k for k, v in _TORCH_OF.items()}


class TgvError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with code {code}: {msg}")
        self.code = code


class NsParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("L", ctypes.c_double * 3), ("gamma", ctypes.c_double),
                ("mach", ctypes.c_double), ("reynolds", ctypes.c_double), ("prandtl", ctypes.c_double),
                ("viscous", ctypes.c_int32), ("split", ctypes.c_int32)]


class NsPrec(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int), ("qt", ctypes.c_int), ("r", ctypes.c_int), ("compute", ctypes.c_int)]


_lib = None
_EXPORTS = {
    "tgv_init": ([ctypes.POINTER(NsParams), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "tgv_init_primitive": ([ctypes.POINTER(NsParams), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                            ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ns_state_from_velocity": ([ctypes.POINTER(NsParams), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ns_state_from_velocity_adjoint": ([ctypes.POINTER(NsParams), ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "dissipation_trapezoid": ([ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                               ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ns_residual": ([ctypes.POINTER(NsParams), ctypes.POINTER(NsPrec), ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.c_void_p], ctypes.c_int),
    "rk_stage": ([ctypes.POINTER(NsParams), ctypes.POINTER(NsPrec), ctypes.c_int, ctypes.c_double,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ns_residual_rk_stage": ([ctypes.POINTER(NsParams), ctypes.POINTER(NsPrec), ctypes.c_int, ctypes.c_double,
                              ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "flow_integrals_workspace_bytes": ([ctypes.POINTER(NsParams)], ctypes.c_size_t),
    "flow_integrals": ([ctypes.POINTER(NsParams), ctypes.POINTER(NsPrec), ctypes.c_void_p, ctypes.c_void_p,
                        ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "flow_integrals_noalloc": ([ctypes.POINTER(NsParams), ctypes.POINTER(NsPrec), ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "ns_residual_adjoint_workspace_bytes": ([ctypes.POINTER(NsParams), ctypes.POINTER(NsPrec)], ctypes.c_size_t),
    "ns_residual_adjoint": ([ctypes.POINTER(NsParams), ctypes.POINTER(NsPrec), ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "rk_stage_adjoint": ([ctypes.POINTER(NsParams), ctypes.POINTER(NsPrec), ctypes.c_int, ctypes.c_double,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "flow_integrals_adjoint_workspace_bytes": ([ctypes.POINTER(NsParams), ctypes.POINTER(NsPrec)],
                                               ctypes.c_size_t),
    "flow_integrals_adjoint": ([ctypes.POINTER(NsParams), ctypes.POINTER(NsPrec), ctypes.c_void_p,
                                ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
                               ctypes.c_int),
    "ns_last_error": ([], ctypes.c_char_p),
    "tgv_abi_version": ([], ctypes.c_int),
}


def load():
    """Load libtgv.so (built by paper_2505_20911_amd/build.py); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2505_20911_amd.build` "
                               "(there is no fallback implementation)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (argt, rest) in _EXPORTS.items():
            fn = getattr(lib, name)
            fn.argtypes = argt
            fn.restype = rest
        _lib = lib
    return _lib


# Split forms of the convective term (ns_split_t).
SPLIT_FORMS = {"blaisdell": 0, "divergence": 1, "feiereisen": 2, "jameson": 3, "kgp": 4, "kok": 5,
               "keep": 6}


@dataclass(frozen=True)
class Params:
    """Grid and physics (paper Sec. 4.1).  n = (nx, ny, nz); split selects the
    convective split form (SPLIT_FORMS)."""
    n: tuple = (32, 32, 32)
    L: tuple = (2 * 3.141592653589793,) * 3
    gamma: float = 1.4
    mach: float = 0.1
    reynolds: float = 1600.0
    prandtl: float = 0.71
    viscous: int = 1
    split: int = 0

    def c(self) -> NsParams:
        p = NsParams()
        for d in range(3):
            p.n[d] = int(self.n[d])
            p.L[d] = float(self.L[d])
        p.gamma, p.mach, p.reynolds, p.prandtl = (float(self.gamma), float(self.mach),
                                                  float(self.reynolds), float(self.prandtl))
        p.viscous = int(self.viscous)
        p.split = int(self.split)
        return p

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (5, nz, ny, nx)

    @property
    def N(self) -> int:
        return int(self.n[0]) * int(self.n[1]) * int(self.n[2])


@dataclass(frozen=True)
class Prec:
    """Storage type of Q, Q~, R and arithmetic type (torch dtypes)."""
    q: torch.dtype = torch.float64
    qt: torch.dtype = torch.float64
    r: torch.dtype = torch.float64
    compute: torch.dtype = torch.float64

    def c(self) -> NsPrec:
        return NsPrec(_CODE_OF[self.q], _CODE_OF[self.qt], _CODE_OF[self.r], _CODE_OF[self.compute])


f64, f32, f16, bf16 = torch.float64, torch.float32, torch.float16, torch.bfloat16
PRESETS = {
    "DP": Prec(f64, f64, f64, f64),
    "SPDP": Prec(f64, f64, f32, f32),
    "SPDP_C64": Prec(f64, f64, f32, f64),
    "SP_DPC": Prec(f32, f32, f32, f64),
    "SP": Prec(f32, f32, f32, f32),
    "HPSP": Prec(f32, f32, f16, f32),
    "HPSP_BF16": Prec(f32, f32, bf16, f32),
    "HP": Prec(f16, f16, f16, f32),
    # per-class variants (Sec. 4.2): "-wk" reduces only the work quantities,
    # here the arithmetic; "-res" only R; "-res+wk" both.  SPDP is SPDP-res+wk,
    # SPDP_C64 SPDP-res, HPSP HPSP-res.
    "SPDP_WK": Prec(f64, f64, f64, f32),
    "HPSP_WK": Prec(f32, f32, f32, f16),
    "HPSP_RESWK": Prec(f32, f32, f16, f16),
    "HP_C16": Prec(f16, f16, f16, f16),
}


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t: torch.Tensor, name: str, dtype=None, numel=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _check(fn: str, rc: int):
    if rc != 0:
        raise TgvError(fn, rc, load().ns_last_error().decode())


def tgv_init(params: Params, q: torch.Tensor, stream=None) -> None:
    code = _CODE_OF.get(q.dtype)
    if code is None:
        raise TypeError(f"unsupported dtype {q.dtype}")
    _check("tgv_init", load().tgv_init(ctypes.byref(params.c()), code, _ptr(q, "q", numel=5 * params.N),
                                       _stream(stream)))


def _code(dtype: torch.dtype) -> int:
    code = _CODE_OF.get(dtype)
    if code is None:
        raise TypeError(f"unsupported dtype {dtype}")
    return code


def tgv_init_primitive(params: Params, u: torch.Tensor, rho: torch.Tensor, p: torch.Tensor, stream=None) -> None:
    N = params.N
    _check("tgv_init_primitive", load().tgv_init_primitive(
        ctypes.byref(params.c()), _code(u.dtype), _ptr(u, "u", u.dtype, 3 * N), _ptr(rho, "rho", u.dtype, N),
        _ptr(p, "p", u.dtype, N), _stream(stream)))


def ns_state_from_velocity(params: Params, u: torch.Tensor, rho: torch.Tensor, p: torch.Tensor, q: torch.Tensor,
                           stream=None) -> None:
    N = params.N
    _check("ns_state_from_velocity", load().ns_state_from_velocity(
        ctypes.byref(params.c()), _code(u.dtype), _ptr(u, "u", u.dtype, 3 * N), _ptr(rho, "rho", u.dtype, N),
        _ptr(p, "p", u.dtype, N), _ptr(q, "q", u.dtype, 5 * N), _stream(stream)))


def ns_state_from_velocity_adjoint(params: Params, u: torch.Tensor, rho: torch.Tensor, q_bar: torch.Tensor,
                                   u_bar: torch.Tensor, stream=None) -> None:
    N = params.N
    _check("ns_state_from_velocity_adjoint", load().ns_state_from_velocity_adjoint(
        ctypes.byref(params.c()), _code(u.dtype), _ptr(u, "u", u.dtype, 3 * N), _ptr(rho, "rho", u.dtype, N),
        _ptr(q_bar, "q_bar", u.dtype, 5 * N), _ptr(u_bar, "u_bar", u.dtype, 3 * N), _stream(stream)))


def dissipation_trapezoid(hist: torch.Tensor, rows: int, dt: float, J: torch.Tensor, stride: int = 8, col: int = 2,
                          stream=None) -> None:
    """J[0] = dt sum_n w_n hist[n, col] over the first `rows` rows (trapezoid weights)."""
    if hist.dim() != 2 or hist.shape[1] != stride or hist.shape[0] < rows:
        raise ValueError(f"hist must be ({rows}+, {stride})")
    _check("dissipation_trapezoid", load().dissipation_trapezoid(
        _ptr(hist, "hist", torch.float64), int(rows), int(stride), int(col), float(dt), _ptr(J, "J", torch.float64, 1),
        _stream(stream)))


def ns_residual(params: Params, prec: Prec, q: torch.Tensor, r: torch.Tensor, stream=None) -> None:
    n5 = 5 * params.N
    _check("ns_residual", load().ns_residual(ctypes.byref(params.c()), ctypes.byref(prec.c()),
                                             _ptr(q, "q", prec.q, n5), _ptr(r, "r", prec.r, n5), _stream(stream)))


def rk_stage(params: Params, prec: Prec, stage: int, dt: float, q: torch.Tensor, qt: torch.Tensor,
             r: torch.Tensor, stream=None) -> None:
    n5 = 5 * params.N
    _check("rk_stage", load().rk_stage(ctypes.byref(params.c()), ctypes.byref(prec.c()), int(stage), float(dt),
                                       _ptr(q, "q", prec.q, n5), _ptr(qt, "qt", prec.qt, n5),
                                       _ptr(r, "r", prec.r, n5), _stream(stream)))


def ns_residual_rk_stage(params: Params, prec: Prec, stage: int, dt: float, q_in: torch.Tensor,
                         q_out: torch.Tensor, qt: torch.Tensor, stream=None) -> None:
    n5 = 5 * params.N
    _check("ns_residual_rk_stage", load().ns_residual_rk_stage(
        ctypes.byref(params.c()), ctypes.byref(prec.c()), int(stage), float(dt), _ptr(q_in, "q_in", prec.q, n5),
        _ptr(q_out, "q_out", prec.q, n5), _ptr(qt, "qt", prec.qt, n5), _stream(stream)))


def flow_integrals_workspace_bytes(params: Params) -> int:
    return int(load().flow_integrals_workspace_bytes(ctypes.byref(params.c())))


def flow_integrals(params: Params, prec: Prec, q: torch.Tensor, workspace: torch.Tensor, out8: torch.Tensor,
                   stream=None) -> None:
    need = flow_integrals_workspace_bytes(params)
    if workspace.numel() * workspace.element_size() < need:
        raise ValueError(f"workspace needs {need} bytes")
    _check("flow_integrals", load().flow_integrals(ctypes.byref(params.c()), ctypes.byref(prec.c()),
                                                   _ptr(q, "q", prec.q, 5 * params.N), _ptr(workspace, "workspace"),
                                                   _ptr(out8, "out8", torch.float64, 8), _stream(stream)))


def flow_integrals_noalloc(params: Params, prec: Prec, q: torch.Tensor, out8: torch.Tensor, stream=None) -> None:
    """flow_integrals without a workspace (the library's static device scratch;
    calls that overlap on one device race)."""
    _check("flow_integrals_noalloc", load().flow_integrals_noalloc(
        ctypes.byref(params.c()), ctypes.byref(prec.c()), _ptr(q, "q", prec.q, 5 * params.N),
        _ptr(out8, "out8", torch.float64, 8), _stream(stream)))


def ns_residual_adjoint_workspace_bytes(params: Params, prec: Prec) -> int:
    return int(load().ns_residual_adjoint_workspace_bytes(ctypes.byref(params.c()), ctypes.byref(prec.c())))


def ns_residual_adjoint(params: Params, prec: Prec, q: torch.Tensor, r_bar: torch.Tensor, q_bar: torch.Tensor,
                        workspace: torch.Tensor, stream=None) -> None:
    n5 = 5 * params.N
    need = ns_residual_adjoint_workspace_bytes(params, prec)
    if workspace.numel() * workspace.element_size() < need:
        raise ValueError(f"workspace needs {need} bytes")
    _check("ns_residual_adjoint", load().ns_residual_adjoint(
        ctypes.byref(params.c()), ctypes.byref(prec.c()), _ptr(q, "q", prec.q, n5), _ptr(r_bar, "r_bar", prec.q, n5),
        _ptr(q_bar, "q_bar", prec.q, n5), _ptr(workspace, "workspace"), _stream(stream)))


def rk_stage_adjoint(params: Params, prec: Prec, stage: int, dt: float, q_bar: torch.Tensor, zeta: torch.Tensor,
                     r_bar: torch.Tensor, stream=None) -> None:
    n5 = 5 * params.N
    _check("rk_stage_adjoint", load().rk_stage_adjoint(
        ctypes.byref(params.c()), ctypes.byref(prec.c()), int(stage), float(dt), _ptr(q_bar, "q_bar", prec.q, n5),
        _ptr(zeta, "zeta", prec.q, n5), _ptr(r_bar, "r_bar", prec.q, n5), _stream(stream)))


def flow_integrals_adjoint_workspace_bytes(params: Params, prec: Prec) -> int:
    return int(load().flow_integrals_adjoint_workspace_bytes(ctypes.byref(params.c()), ctypes.byref(prec.c())))


def flow_integrals_adjoint(params: Params, prec: Prec, q: torch.Tensor, eps_bar: float, q_bar: torch.Tensor,
                           workspace: torch.Tensor, stream=None) -> None:
    n5 = 5 * params.N
    need = flow_integrals_adjoint_workspace_bytes(params, prec)
    if workspace.numel() * workspace.element_size() < need:
        raise ValueError(f"workspace needs {need} bytes")
    _check("flow_integrals_adjoint", load().flow_integrals_adjoint(
        ctypes.byref(params.c()), ctypes.byref(prec.c()), _ptr(q, "q", prec.q, n5), float(eps_bar),
        _ptr(q_bar, "q_bar", prec.q, n5), _ptr(workspace, "workspace"), _stream(stream)))


def ns_last_error() -> str:
    return load().ns_last_error().decode()


def tgv_abi_version() -> int:
    return int(load().tgv_abi_version())
