"""The adjoint workload at full size: Taylor-Green 128^3, 400 RK3 steps
(dt = 9.25e-4), revolve checkpointing with 20 snapshot buffers.  The gradient
of the time-integrated dissipation J = dt sum_n w_n eps^S(Q^n) with respect to
the initial velocity (density and pressure held fixed) is checked against
central finite differences, eps = 1e-6, along 8 seeded unnormalised Gaussian
directions (FP64 form), and the FP32 form's gradient against the FP64 one."""
import sys
import time

import numpy as np
import pytest
import torch

import tgv_synth as S
from paper_2505_20911_amd import tgv
from paper_2505_20911_amd.adjoint import CheckpointedDissipation, dissipation, state_from_velocity

pytestmark = pytest.mark.gpu
DEV = "cuda"
N, STEPS, DT, SLOTS = 128, 400, 9.25e-4, 20


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    p = tgv.Params(n=(N, N, N))
    q0 = torch.empty(p.shape, dtype=torch.float64, device=DEV)
    tgv.tgv_init(p, q0)
    rho0 = q0[0].clone()
    u0 = (q0[1:4] / rho0).clone()
    p0 = (q0[4] - 0.5 * rho0 * (u0 * u0).sum(0)) * (p.gamma - 1.0)
    t = time.perf_counter()
    uu = u0.clone().requires_grad_(True)
    J = dissipation(state_from_velocity(uu, rho0, p0, p.gamma), p, tgv.PRESETS["DP"], DT, STEPS, slots=SLOTS)
    J.backward()
    torch.cuda.synchronize()
    say("FP64 J", float(J.detach()), "forward+reverse", time.perf_counter() - t, "s")
    return p, u0, rho0, p0, uu.grad.detach(), float(J.detach())


def test_revolve_schedule_cost():
    from paper_2505_20911_amd import revolve
    assert revolve.optimal_advances(STEPS, SLOTS) == revolve.binomial_closed_form(STEPS, SLOTS) == 924


def test_gradient_matches_central_differences(setup):
    p, u0, rho0, p0, g, J = setup
    runner = CheckpointedDissipation(p, tgv.PRESETS["DP"], DT, STEPS, slots=SLOTS)
    eps = 1e-6
    worst = 0.0
    for s in range(8):
        d = torch.from_numpy(S.directions(p.n, s)).to(DEV)
        Jp = runner.forward(state_from_velocity(u0 + eps * d, rho0, p0, p.gamma))
        Jm = runner.forward(state_from_velocity(u0 - eps * d, rho0, p0, p.gamma))
        fd = (Jp - Jm) / (2 * eps)
        ad = float((g * d).sum())
        rel = abs(fd - ad) / abs(ad)
        worst = max(worst, rel)
        say(f"direction {s}: FD {fd:.12e} adjoint {ad:.12e} rel {rel:.2e}")
    assert worst <= 1e-6


def test_fp32_gradient_close_to_fp64(setup):
    p, u0, rho0, p0, g64, J64 = setup
    prec = tgv.PRESETS["SP"]
    uu = u0.float().clone().requires_grad_(True)
    J = dissipation(state_from_velocity(uu, rho0.float(), p0.float(), p.gamma), p, prec, DT, STEPS, slots=SLOTS)
    J.backward()
    g32 = uu.grad.detach().double()
    rel = float(torch.linalg.vector_norm(g32 - g64) / torch.linalg.vector_norm(g64))
    say("FP32 J", float(J.detach()), "FP64 J", J64, "gradient rel L2 difference", rel)
    assert abs(float(J.detach()) - J64) <= 1e-4 * abs(J64)
    assert rel <= 1e-2


def test_fd_step_sits_on_the_plateau(setup):
    """Central differences along direction 0 for eps = 1e-4 .. 1e-8: the
    truncation error (O(eps^2)) falls and the rounding error (O(u J / eps))
    rises; eps = 1e-6 and 1e-5 both sit on the plateau between them."""
    p, u0, rho0, p0, g, J = setup
    runner = CheckpointedDissipation(p, tgv.PRESETS["DP"], DT, STEPS, slots=SLOTS)
    d = torch.from_numpy(S.directions(p.n, 0)).to(DEV)
    ad = float((g * d).sum())
    rel = {}
    for eps in (1e-4, 1e-5, 1e-6, 1e-7, 1e-8):
        Jp = runner.forward(state_from_velocity(u0 + eps * d, rho0, p0, p.gamma))
        Jm = runner.forward(state_from_velocity(u0 - eps * d, rho0, p0, p.gamma))
        rel[eps] = abs((Jp - Jm) / (2 * eps) - ad) / abs(ad)
        say(f"eps {eps:.0e}: relative FD - adjoint difference {rel[eps]:.2e}")
    assert rel[1e-5] <= 1e-6 and rel[1e-6] <= 1e-6
