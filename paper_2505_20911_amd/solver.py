"""Time-stepping driver over the C-ABI: owns Q, Q~, R and the integrals
workspace on one GPU and enqueues the step (paper Sec. 3.1: per RK stage one
residual evaluation then the two-register update) on one stream.  History
samples of the integrals stay on the device until read.

fused=True (default) uses ns_residual_rk_stage: each stage is one pass that
reads Q from one buffer and writes the advanced Q to the other (the stencil
must see the old Q around every point), so Q ping-pongs between two buffers
and R is never stored.  fused=False calls ns_residual then rk_stage."""
from __future__ import annotations

import torch

from . import tgv
from .tgv import Params, Prec


class TGVSolver:
    def __init__(self, params: Params, prec: Prec, device="cuda", stream=None, fused: bool = True):
        self.params = params
        self.prec = prec
        self.device = torch.device(device)
        self.stream = stream
        self.fused = fused
        shape = params.shape
        self._q = [torch.empty(shape, dtype=prec.q, device=self.device)]
        if fused:
            self._q.append(torch.empty(shape, dtype=prec.q, device=self.device))
            self.r = None
        else:
            self.r = torch.empty(shape, dtype=prec.r, device=self.device)
        self._cur = 0
        self.qt = torch.zeros(shape, dtype=prec.qt, device=self.device)
        nbytes = tgv.flow_integrals_workspace_bytes(params)
        self.work = torch.empty((nbytes + 7) // 8, dtype=torch.float64, device=self.device)

    @property
    def q(self) -> torch.Tensor:
        """The current state Q."""
        return self._q[self._cur]

    def init(self) -> None:
        tgv.tgv_init(self.params, self.q, self.stream)

    def stage(self, i: int, dt: float) -> None:
        if self.fused:
            tgv.ns_residual_rk_stage(self.params, self.prec, i, dt, self._q[self._cur], self._q[1 - self._cur],
                                     self.qt, self.stream)
            self._cur = 1 - self._cur
        else:
            tgv.ns_residual(self.params, self.prec, self.q, self.r, self.stream)
            tgv.rk_stage(self.params, self.prec, i, dt, self.q, self.qt, self.r, self.stream)

    def step(self, dt: float) -> None:
        for i in range(3):
            self.stage(i, dt)

    def integrals(self, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(8, dtype=torch.float64, device=self.device)
        tgv.flow_integrals(self.params, self.prec, self.q, self.work, out, self.stream)
        return out

    def run(self, nsteps: int, dt: float, every: int = 0) -> torch.Tensor | None:
        """Advance nsteps steps; with every > 0 returns a device tensor of
        integrals rows after 0, every, 2*every, ... steps."""
        hist = None
        if every > 0:
            hist = torch.empty((nsteps // every + 1, 8), dtype=torch.float64, device=self.device)
        row = 0
        for n in range(nsteps + 1):
            if hist is not None and n % every == 0:
                self.integrals(hist[row])
                row += 1
            if n == nsteps:
                break
            self.step(dt)
        return hist
