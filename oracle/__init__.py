"""FP64 CPU oracle for the TGV explicit time step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it, and it shares no code
with that path.

What it computes (paper: Sec. 2.3.1 scheme and split forms, Sec. 3.1 state
vector and two-register Runge-Kutta update, Sec. 4.1 Taylor-Green initial
condition and the K / eps^S integrals) is implemented in plain C++ loops in
``tgv_oracle.cpp``; this module is ctypes marshalling plus a pure-NumPy dense
circulant evaluation (``brute``) for tiny grids.  The readings it takes where
the paper is silent are listed at the top of ``tgv_oracle.cpp``.

Arrays are float64 (or complex128), C-contiguous, shaped (5, nz, ny, nx) for
the conserved vector Q = (rho, rho u, rho v, rho w, rho E), x fastest.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtgv_oracle.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    sigs = {
        "oracle_init": [dp, dp],
        "oracle_residual": [dp, dp, dp],
        "oracle_residual_c": [dp, dp, dp],
        "oracle_residual_adjoint": [dp, dp, dp, dp],
        "oracle_rk_stage": [ctypes.c_int, ctypes.c_double, ctypes.c_long, dp, dp, dp],
        "oracle_rk_stage_c": [ctypes.c_int, ctypes.c_double, ctypes.c_long, dp, dp, dp],
        "oracle_integrals": [dp, dp, dp],
        "oracle_integrals_c": [dp, dp, dp],
        "oracle_integrals_adjoint": [dp, dp, ctypes.c_double, dp],
        "oracle_residual_at": [dp, dp, ctypes.c_long, ctypes.POINTER(ctypes.c_long), dp],
        "oracle_init_at": [dp, ctypes.c_long, ctypes.POINTER(ctypes.c_long), dp],
        "oracle_d1": [dp, dp, ctypes.c_int, dp],
        "oracle_d2": [dp, dp, ctypes.c_int, dp],
        "oracle_run": [dp, ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp],
        "oracle_run_c": [dp, ctypes.c_double, ctypes.c_int, dp],
        "oracle_dissipation_c": [dp, ctypes.c_double, ctypes.c_int, dp, dp],
        "oracle_dissipation_grad": [dp, ctypes.c_double, ctypes.c_int, dp, dp, dp],
    }
    for name, argt in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = argt
        fn.restype = ctypes.c_int if name in _RETURNS_STATUS else None
    _lib = lib
    return lib


# Entry points that return a status (0, or -1 when they refuse the split form).
_RETURNS_STATUS = ("oracle_residual_adjoint", "oracle_dissipation_grad")


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# Split forms of the convective term (Sec. 2.3.1 and the inviscid comparison of
# Sec. 4.2), by the value of Params.split.
SPLIT_FORMS = {"blaisdell": 0, "divergence": 1, "feiereisen": 2, "jameson": 3, "kgp": 4, "kok": 5, "keep": 6}


def _blaisdell_only(status, what):
    """The C routine refuses split forms other than Blaisdell (status -1)."""
    if status != 0:
        raise ValueError(f"{what} is written for the Blaisdell split form only")


@dataclass
class Params:
    """Physical and grid parameters (Sec. 4.1).  n = (nx, ny, nz)."""
    n: tuple = (32, 32, 32)
    L: tuple = (2 * np.pi, 2 * np.pi, 2 * np.pi)
    gamma: float = 1.4
    mach: float = 0.1
    re: float = 1600.0
    pr: float = 0.71
    viscous: int = 1
    split: int = 0  # convective split form, SPLIT_FORMS

    def packed(self) -> np.ndarray:
        return np.array(list(self.n) + list(self.L) +
                        [self.gamma, self.mach, self.re, self.pr, float(self.viscous), float(self.split)],
                        dtype=np.float64)

    @property
    def shape(self):
        nx, ny, nz = self.n
        return (5, nz, ny, nx)

    @property
    def N(self) -> int:
        return int(np.prod(self.n))

    def h(self, d: int) -> float:
        return self.L[d] / self.n[d]


def _q(P: Params, q, dtype=np.float64) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=dtype)
    assert q.shape == P.shape, (q.shape, P.shape)
    return q


def init(P: Params) -> np.ndarray:
    """Taylor-Green initial state (Sec. 4.1 initial-condition equations)."""
    q = np.empty(P.shape, np.float64)
    _load().oracle_init(_p(P.packed()), _p(q))
    return q


def residual(P: Params, q) -> np.ndarray:
    """R = dQ/dt (Sec. 3.1: the residual holding all remaining terms)."""
    q = _q(P, q)
    r = np.empty_like(q)
    _load().oracle_residual(_p(P.packed()), _p(q), _p(r))
    return r


def residual_c(P: Params, q) -> np.ndarray:
    """The same residual evaluated in complex arithmetic (complex-step checks)."""
    q = _q(P, q, np.complex128)
    r = np.empty_like(q)
    _load().oracle_residual_c(_p(P.packed()), q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return r


def residual_adjoint(P: Params, q, rbar, qbar=None) -> np.ndarray:
    """qbar += (dR/dQ)^T rbar (hand-written reverse mode of ``residual``)."""
    q = _q(P, q)
    rbar = _q(P, rbar)
    if qbar is None:
        qbar = np.zeros_like(q)
    _blaisdell_only(_load().oracle_residual_adjoint(_p(P.packed()), _p(q), _p(rbar), _p(qbar)),
                    "residual_adjoint")
    return qbar


RK_A = (0.0, -5.0 / 9.0, -153.0 / 128.0)
RK_B = (1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0)


def rk_stage(stage: int, dt: float, q: np.ndarray, qt: np.ndarray, r: np.ndarray) -> None:
    """In place: Qt <- A_i Qt + dt R ; Q <- Q + B_i Qt (Sec. 3.1 update equations)."""
    for a in (q, qt, r):
        assert a.flags.c_contiguous and a.dtype in (np.float64, np.complex128)
    assert q.dtype == qt.dtype == r.dtype and q.size == qt.size == r.size
    lib = _load()
    if q.dtype == np.complex128:
        lib.oracle_rk_stage_c(stage, dt, q.size, q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              qt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                              r.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    else:
        lib.oracle_rk_stage(stage, dt, q.size, _p(q), _p(qt), _p(r))


INTEGRAL_NAMES = ("K", "K_rho", "eps_S", "mean_rho", "mean_m1", "mean_m2", "mean_m3", "mean_E")


def integrals(P: Params, q) -> np.ndarray:
    """[K, K_rho, eps^S, <rho>, <m1>, <m2>, <m3>, <rho E>] (Sec. 4.1 K and eps^S equations)."""
    q = _q(P, q)
    out = np.empty(8, np.float64)
    _load().oracle_integrals(_p(P.packed()), _p(q), _p(out))
    return out


def integrals_c(P: Params, q) -> np.ndarray:
    q = _q(P, q, np.complex128)
    out = np.empty(8, np.complex128)
    _load().oracle_integrals_c(_p(P.packed()), q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def integrals_adjoint(P: Params, q, eps_bar: float, qbar=None) -> np.ndarray:
    """qbar += eps_bar * d(eps^S)/dQ."""
    q = _q(P, q)
    if qbar is None:
        qbar = np.zeros_like(q)
    _load().oracle_integrals_adjoint(_p(P.packed()), _p(q), float(eps_bar), _p(qbar))
    return qbar


def d1(P: Params, f, axis: int) -> np.ndarray:
    """4th-order central first derivative of a scalar field along axis (0=x, 1=y, 2=z)."""
    f = np.ascontiguousarray(f, np.float64)
    assert f.shape == P.shape[1:]
    out = np.empty_like(f)
    _load().oracle_d1(_p(P.packed()), _p(f), axis, _p(out))
    return out


def d2(P: Params, f, axis: int) -> np.ndarray:
    f = np.ascontiguousarray(f, np.float64)
    assert f.shape == P.shape[1:]
    out = np.empty_like(f)
    _load().oracle_d2(_p(P.packed()), _p(f), axis, _p(out))
    return out


def run(P: Params, dt: float, nsteps: int, q=None, every: int = 0):
    """Advance nsteps RK3 steps.  Returns (Q, history) with history[m] the
    integrals after m*every steps (None when every == 0)."""
    q = init(P) if q is None else _q(P, q).copy()
    hist = None
    hp = None
    if every > 0:
        hist = np.zeros((nsteps // every + 1, 8), np.float64)
        hp = _p(hist)
    _load().oracle_run(_p(P.packed()), float(dt), int(nsteps), int(every), _p(q), hp)
    return q, hist


def run_c(P: Params, dt: float, nsteps: int, q) -> np.ndarray:
    q = _q(P, q, np.complex128).copy()
    _load().oracle_run_c(_p(P.packed()), float(dt), int(nsteps),
                         q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return q


def dissipation_c(P: Params, dt: float, nsteps: int, q0) -> complex:
    """J = dt * sum_n w_n eps^S(Q^n), trapezoid weights, complex arithmetic."""
    q = _q(P, q0, np.complex128).copy()
    J = np.zeros(1, np.complex128)
    _load().oracle_dissipation_c(_p(P.packed()), float(dt), int(nsteps),
                                 q.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 J.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return complex(J[0])


def dissipation_grad(P: Params, dt: float, nsteps: int, q0):
    """(J, dJ/dQ^0) by store-all reverse mode through the RK3 stages."""
    q0 = _q(P, q0)
    J = np.zeros(1, np.float64)
    g = np.zeros_like(q0)
    _blaisdell_only(_load().oracle_dissipation_grad(_p(P.packed()), float(dt), int(nsteps), _p(q0), _p(J), _p(g)),
                    "dissipation_grad")
    return float(J[0]), g


def init_primitive(P: Params):
    """Taylor-Green initial fields in primitive form (Sec. 4.1 initial
    condition, isothermal density rho = gamma M^2 p), FP64:
    u (3, nz, ny, nx), rho and p (nz, ny, nx).  Plain NumPy on the grid
    x_i = i L / n."""
    nx, ny, nz = P.n
    x = np.arange(nx) * (P.L[0] / nx)
    y = np.arange(ny) * (P.L[1] / ny)
    z = np.arange(nz) * (P.L[2] / nz)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    u = np.empty((3, nz, ny, nx))
    u[0] = np.sin(X) * np.cos(Y) * np.cos(Z)
    u[1] = -np.cos(X) * np.sin(Y) * np.cos(Z)
    u[2] = 0.0
    gm2 = P.gamma * P.mach ** 2
    p = 1.0 / gm2 + (np.cos(2 * X) + np.cos(2 * Y)) * (2.0 + np.cos(2 * Z)) / 16.0
    return u, gm2 * p, p


def velocity_ic_state(P: Params, u0: np.ndarray, rho0: np.ndarray, p0: np.ndarray) -> np.ndarray:
    """Q^0 built from a velocity field u0 (3, nz, ny, nx) with the density and
    pressure fields held fixed: m = rho0 u0, rho E = p0/(gamma-1) + 1/2 rho0 |u0|^2."""
    q = np.empty(P.shape, np.result_type(u0, rho0, p0, np.float64))
    q[0] = rho0
    q[1:4] = rho0[None] * u0
    q[4] = p0 / (P.gamma - 1.0) + 0.5 * rho0 * (u0 ** 2).sum(axis=0)
    return q


def velocity_grad_from_state_grad(P: Params, qbar0: np.ndarray, u0: np.ndarray,
                                  rho0: np.ndarray) -> np.ndarray:
    """Chain rule of ``velocity_ic_state``: dJ/du0_a = rho0 qbar_{m_a} + rho0 u0_a qbar_E."""
    return rho0[None] * qbar0[1:4] + rho0[None] * u0 * qbar0[4][None]


def residual_at(P: Params, q, idx) -> np.ndarray:
    """Residual at the listed linear point indices (pointwise evaluation, every
    split form), shape (len(idx), 5)."""
    q = _q(P, q)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((idx.size, 5), np.float64)
    _load().oracle_residual_at(_p(P.packed()), _p(q), idx.size,
                               idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _p(out))
    return out


def init_at(P: Params, idx) -> np.ndarray:
    """Initial state at the listed linear point indices, shape (len(idx), 5)."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((idx.size, 5), np.float64)
    _load().oracle_init_at(_p(P.packed()), idx.size,
                           idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _p(out))
    return out
