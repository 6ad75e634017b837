"""Gradient of the time-integrated dissipation with respect to the initial
state, by the discrete adjoint of the RK3 time step with binomial
checkpointing, exposed as a ``torch.autograd.Function``.

Objective (trapezoid rule over the step boundaries, eps^S as in Sec. 4.1):
    J = dt * sum_{n=0}^{l} w_n eps^S(Q^n),   w_0 = w_l = 1/2, else 1.
Reverse of one step (Sec. 3.1 update, read backwards): with stage inputs
Y_0 = Q^{n-1}, Y_1, Y_2 re-taped from the restored state and zeta = 0,
for i = 2, 1, 0:  zeta += B_i Q_bar ; R_bar = dt zeta ; zeta <- A_i zeta ;
Q_bar += (dR/dQ)(Y_i)^T R_bar   (rk_stage_adjoint, ns_residual_adjoint),
then Q_bar += dt w_{n-1} d(eps^S)/dQ(Y_0)   (flow_integrals_adjoint).
The control is the initial velocity u0 with density and pressure held fixed:
Q^0 = (rho0, rho0 u0, p0/(gamma-1) + rho0 |u0|^2 / 2) (ns_state_from_velocity),
and dJ/du0 = rho0 (Q_bar_m + u0 Q_bar_E) (ns_state_from_velocity_adjoint).
Every arithmetic step -- the state map, the time steps, the integrals, their
adjoints and the trapezoid sum J -- runs in libtgv's kernels; this module
sequences the calls and the snapshot copies.
"""
from __future__ import annotations

import torch

from . import revolve, tgv
from .tgv import Params, Prec


def state_from_velocity(u0: torch.Tensor, rho0: torch.Tensor, p0: torch.Tensor, params: Params) -> torch.Tensor:
    """Q^0 (5, nz, ny, nx) from a velocity field (3, nz, ny, nx) at fixed
    density and pressure (ns_state_from_velocity), in u0's dtype."""
    q = torch.empty(params.shape, dtype=u0.dtype, device=u0.device)
    tgv.ns_state_from_velocity(params, u0.detach().contiguous(), rho0.contiguous(), p0.contiguous(), q)
    return q


def taylor_green_primitive(params: Params, dtype=torch.float64, device="cuda"):
    """(u0, rho0, p0) of the Taylor-Green initial state (tgv_init_primitive)."""
    nx, ny, nz = params.n
    u = torch.empty((3, nz, ny, nx), dtype=dtype, device=device)
    rho = torch.empty((nz, ny, nx), dtype=dtype, device=device)
    p = torch.empty((nz, ny, nx), dtype=dtype, device=device)
    tgv.tgv_init_primitive(params, u, rho, p)
    return u, rho, p


class CheckpointedDissipation:
    """Forward sweep and revolve-scheduled reverse sweep on one GPU."""

    def __init__(self, params: Params, prec: Prec, dt: float, nsteps: int, slots: int = 20, device="cuda"):
        if prec.q != prec.qt or prec.q != prec.r or prec.q != prec.compute:
            raise ValueError("the adjoint runs with a single storage/compute type (DP or SP preset)")
        self.params, self.prec, self.dt, self.l = params, prec, float(dt), int(nsteps)
        self.slots = min(int(slots), max(self.l - 1, 0))
        self.device = torch.device(device)
        shape, dt_ = params.shape, prec.q
        mk = lambda: torch.empty(shape, dtype=dt_, device=self.device)
        # Forward steps run the fused residual + stage kernel, ping-ponging
        # between `cur` and `alt`; Q~ is updated in place.
        self.cur, self.alt, self.qt = mk(), mk(), torch.zeros(shape, dtype=dt_, device=self.device)
        self.Y = [None, mk(), mk()]  # stage inputs of the step being reversed (Y[0] is `cur`)
        self.qbar, self.zeta, self.rbar = mk(), mk(), mk()
        self.snap = [mk() for _ in range(self.slots)]
        self.qlast = mk()
        nb = tgv.flow_integrals_workspace_bytes(params)
        self.iwork = torch.empty((nb + 7) // 8, dtype=torch.float64, device=self.device)
        self.awork = torch.empty(tgv.ns_residual_adjoint_workspace_bytes(params, prec) // 8 + 1,
                                 dtype=torch.float64, device=self.device)
        self.ewrk = torch.empty(tgv.flow_integrals_adjoint_workspace_bytes(params, prec) // 8 + 1,
                                dtype=torch.float64, device=self.device)
        self.eps = torch.zeros((self.l + 1, 8), dtype=torch.float64, device=self.device)
        self.J = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.actions = revolve.schedule(self.l, self.slots) if self.l > 0 else []
        self.advances = 0

    def weight(self, n: int) -> float:
        return 0.5 if n in (0, self.l) else 1.0

    # -- forward pieces
    def _stage(self, i: int, q_in: torch.Tensor, q_out: torch.Tensor) -> None:
        tgv.ns_residual_rk_stage(self.params, self.prec, i, self.dt, q_in, q_out, self.qt)

    def _step(self, q: torch.Tensor) -> torch.Tensor:
        """One RK3 step from q (left unchanged only if it is not `alt`);
        returns the buffer that holds the result, which is `alt` on entry."""
        a, b = q, self.alt
        self._stage(0, a, b)
        self._stage(1, b, a)
        self._stage(2, a, b)
        self.alt = a
        self.advances += 1
        return b

    def _advance(self) -> None:
        self.cur = self._step(self.cur)

    def _integrals(self, q: torch.Tensor, n: int) -> None:
        tgv.flow_integrals(self.params, self.prec, q, self.iwork, self.eps[n])

    def _slot(self, s: int, q0: torch.Tensor) -> torch.Tensor:
        return q0 if s < 0 else self.snap[s]

    def forward(self, q0: torch.Tensor) -> float:
        """Runs the schedule's first descent (storing its snapshots) and one
        extra step to Q^l; returns J (synchronising on it)."""
        return float(self.forward_device(q0)[0])

    def forward_device(self, q0: torch.Tensor) -> torch.Tensor:
        """As forward, returning J as a one-element device tensor (no host sync)."""
        self.cur.copy_(q0)
        self._integrals(self.cur, 0)
        n = 0
        self._pos = 0
        for k, act in enumerate(self.actions):
            if act[0] == "reverse":
                self._pos = k
                break
            if act[0] == "advance":
                self._advance()
                n += 1
                self._integrals(self.cur, n)
            elif act[0] == "store":
                self.snap[act[1]].copy_(self.cur)
            elif act[0] in ("restore", "free"):  # cannot occur before the first reversal
                raise AssertionError(act)
        if self.l > 0:
            # Q^{l-1} -> Q^l in `qlast` for eps^S(Q^l), keeping Q^{l-1} in `cur`
            self.qlast.copy_(self.cur)
            self.qlast = self._step(self.qlast)
            self._integrals(self.qlast, self.l)
        # J = dt sum_n w_n eps^S(Q^n), trapezoid weights (with l = 0 the one
        # row has weight 1/2, as the reverse sweep's seed)
        tgv.dissipation_trapezoid(self.eps, self.l + 1, self.dt, self.J)
        return self.J

    # -- reverse pieces
    def _reverse_step(self, n: int, scale: float) -> None:
        """Reverse step n; the current state is Q^{n-1}.  Only the stage
        inputs Y_0 = Q^{n-1}, Y_1, Y_2 are needed (not Q^n), and the schedule
        restores a snapshot after every reversal, so `cur` is left at Q^{n-1}."""
        self.Y[0] = self.cur
        self._stage(0, self.Y[0], self.Y[1])
        self._stage(1, self.Y[1], self.Y[2])
        for i in (2, 1, 0):
            tgv.rk_stage_adjoint(self.params, self.prec, i, self.dt, self.qbar, self.zeta, self.rbar)
            tgv.ns_residual_adjoint(self.params, self.prec, self.Y[i], self.rbar, self.qbar, self.awork)
        tgv.flow_integrals_adjoint(self.params, self.prec, self.Y[0], scale * self.dt * self.weight(n - 1),
                                   self.qbar, self.ewrk)

    def backward(self, q0: torch.Tensor, scale: float = 1.0) -> torch.Tensor:
        """Returns scale * dJ/dQ^0 (a new tensor)."""
        self.qbar.zero_()
        self.zeta.zero_()
        if self.l == 0:
            tgv.flow_integrals_adjoint(self.params, self.prec, q0, scale * self.dt * self.weight(0), self.qbar,
                                       self.ewrk)
            return self.qbar.clone()
        tgv.flow_integrals_adjoint(self.params, self.prec, self.qlast, scale * self.dt * self.weight(self.l),
                                   self.qbar, self.ewrk)
        for act in self.actions[self._pos:]:
            kind = act[0]
            if kind == "advance":
                self._advance()
            elif kind == "store":
                self.snap[act[1]].copy_(self.cur)
            elif kind == "restore":
                self.cur.copy_(self._slot(act[1], q0))
            elif kind == "reverse":
                self._reverse_step(act[1], scale)
        return self.qbar.clone()


class TGVDissipation(torch.autograd.Function):
    """J(u0) = dt sum_n w_n eps^S(Q^n) over `nsteps` RK3 steps from
    Q^0 = state_from_velocity(u0, rho0, p0); backward returns dJ/du0 through
    the discrete adjoint with revolve checkpointing and the adjoint of the
    state map (rho0 and p0 are held fixed and get no gradient)."""

    @staticmethod
    def forward(ctx, u0: torch.Tensor, rho0: torch.Tensor, p0: torch.Tensor, runner: CheckpointedDissipation):
        u0c = u0.detach().contiguous()
        rho0c = rho0.detach().contiguous()
        q0 = state_from_velocity(u0c, rho0c, p0.detach(), runner.params)
        J = runner.forward_device(q0)
        ctx.runner = runner
        ctx.save_for_backward(q0, u0c, rho0c)
        return J[0].clone()

    @staticmethod
    def backward(ctx, gJ):
        q0, u0, rho0 = ctx.saved_tensors
        qbar = ctx.runner.backward(q0, float(gJ))
        ubar = torch.empty_like(u0)
        tgv.ns_state_from_velocity_adjoint(ctx.runner.params, u0, rho0, qbar, ubar)
        return ubar, None, None, None


def dissipation(u0: torch.Tensor, rho0: torch.Tensor, p0: torch.Tensor, params: Params, prec: Prec, dt: float,
                nsteps: int, slots: int = 20) -> torch.Tensor:
    """J(u0) as a differentiable scalar (TGVDissipation)."""
    runner = CheckpointedDissipation(params, prec, dt, nsteps, slots, device=u0.device)
    return TGVDissipation.apply(u0, rho0, p0, runner)
