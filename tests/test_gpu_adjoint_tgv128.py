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
from paper_2505_20911_amd.adjoint import (CheckpointedDissipation, dissipation, state_from_velocity,
                                          taylor_green_primitive)

pytestmark = pytest.mark.gpu
DEV = "cuda"
N, STEPS, DT, SLOTS = 128, 400, 9.25e-4, 20


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    p = tgv.Params(n=(N, N, N))
    u0, rho0, p0 = taylor_green_primitive(p)
    t = time.perf_counter()
    uu = u0.clone().requires_grad_(True)
    J = dissipation(uu, rho0, p0, p, tgv.PRESETS["DP"], DT, STEPS, slots=SLOTS)
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
        Jp = runner.forward(state_from_velocity(u0 + eps * d, rho0, p0, p))
        Jm = runner.forward(state_from_velocity(u0 - eps * d, rho0, p0, p))
        fd = (Jp - Jm) / (2 * eps)
        ad = float((g * d).sum())
        rel = abs(fd - ad) / abs(ad)
        worst = max(worst, rel)
        say(f"direction {s}: FD {fd:.12e} adjoint {ad:.12e} rel {rel:.2e}")
    assert worst <= 1e-6


def test_fp32_gradient_close_to_fp64(setup):
    """The FP32 form's gradient against the FP64 one.  Bound: every one of the
    6 * STEPS stage evaluations (3 per step forward, 3 reversed) perturbs the
    result by at most eps_stage relative, the FP32 rounding bound of one
    residual adjoint (64 u on the adjoint term scale, as in the element-wise
    SP test) over the adjoint's magnitude, measured at the initial state with
    a seeded R_bar; independent roundings accumulate as a random walk, so by
    the probabilistic rounding-error bound of Higham and Mary (2019) the
    relative error stays below lambda sqrt(6 STEPS) eps_stage with
    probability >= 1 - 2 exp(-lambda^2 / 2); lambda = 4."""
    import numpy as np
    from tgv_testutil import UNIT_ROUNDOFF, adjoint_term_scale
    p, u0, rho0, p0, g64, J64 = setup
    prec = tgv.PRESETS["SP"]
    # per-stage rounding bound at the initial state
    q0 = state_from_velocity(u0, rho0, p0, p)
    rbar = torch.from_numpy(S.random_field(p.shape, 21)).to(DEV)
    qb = torch.zeros_like(q0)
    aw = torch.empty(tgv.ns_residual_adjoint_workspace_bytes(p, tgv.PRESETS["DP"]) // 8 + 1, dtype=torch.float64,
                     device=DEV)
    tgv.ns_residual_adjoint(p, tgv.PRESETS["DP"], q0, rbar, qb, aw)
    scale = adjoint_term_scale(p, q0.cpu().numpy(), rbar.cpu().numpy())
    eps_stage = 64 * UNIT_ROUNDOFF[torch.float32] * scale / float(qb.abs().max())
    bound = 4.0 * np.sqrt(6 * STEPS) * eps_stage
    del q0, rbar, qb, aw
    u32, rho32, p32 = taylor_green_primitive(p, torch.float32)
    uu = u32.clone().requires_grad_(True)
    J = dissipation(uu, rho32, p32, p, prec, DT, STEPS, slots=SLOTS)
    J.backward()
    g32 = uu.grad.detach().double()
    rel = float(torch.linalg.vector_norm(g32 - g64) / torch.linalg.vector_norm(g64))
    relJ = abs(float(J.detach()) - J64) / abs(J64)
    say("FP32 J", float(J.detach()), "FP64 J", J64, "rel", relJ, "gradient rel L2 difference", rel,
        "per-stage bound", eps_stage, "bound", bound)
    assert relJ <= bound
    assert rel <= bound


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
        Jp = runner.forward(state_from_velocity(u0 + eps * d, rho0, p0, p))
        Jm = runner.forward(state_from_velocity(u0 - eps * d, rho0, p0, p))
        rel[eps] = abs((Jp - Jm) / (2 * eps) - ad) / abs(ad)
        say(f"eps {eps:.0e}: relative FD - adjoint difference {rel[eps]:.2e}")
    assert rel[1e-5] <= 1e-6 and rel[1e-6] <= 1e-6
