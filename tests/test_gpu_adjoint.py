"""GPU parity of the discrete adjoint: kernels against the oracle's own
hand-written FP64 adjoint (itself pinned by complex step), checkpointed
against store-all reverse sweeps, and the autograd gradient against central
finite differences."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import tgv_synth as S
from paper_2505_20911_amd import tgv
from paper_2505_20911_amd.adjoint import CheckpointedDissipation, TGVDissipation, dissipation, state_from_velocity
from tgv_testutil import oracle_params, widened

pytestmark = pytest.mark.gpu
DEV = "cuda"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def work_for(p, prec, fn):
    nbytes = fn(p, prec)
    return torch.empty(nbytes // 8 + 1, dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("n", [(12, 16, 10), (16, 16, 16), (5, 6, 7)])
@pytest.mark.parametrize("kind", ["tgv", "smooth", "noise"])
@pytest.mark.parametrize("viscous", [1, 0])
def test_residual_adjoint_dp_matches_oracle(n, kind, viscous):
    say("adjoint DP", n, kind, viscous)
    p = tgv.Params(n=n, viscous=viscous)
    q64 = O.init(oracle_params(p)) if kind == "tgv" else S.random_state(n, 5, smooth=(kind == "smooth"))
    rbar = S.random_field(p.shape, 6)
    qb0 = S.random_field(p.shape, 7)  # accumulate into a non-zero q_bar
    ref = O.residual_adjoint(oracle_params(p), q64, rbar, qb0.copy())
    prec = tgv.PRESETS["DP"]
    qb = torch.from_numpy(qb0).to(DEV)
    tgv.ns_residual_adjoint(p, prec, torch.from_numpy(q64).to(DEV), torch.from_numpy(rbar).to(DEV), qb,
                            work_for(p, prec, tgv.ns_residual_adjoint_workspace_bytes))
    got = qb.cpu().numpy()
    scale = np.abs(ref - qb0).reshape(5, -1).max(1)
    err = np.abs(got - ref).reshape(5, -1).max(1)
    say("  err / max|adjoint|", err / scale)
    assert np.all(err <= 1e-11 * scale), err / scale


def test_residual_adjoint_sp_within_rounding():
    n = (12, 16, 10)
    p = tgv.Params(n=n)
    q32 = torch.from_numpy(S.random_state(n, 5, smooth=True)).float()
    r32 = torch.from_numpy(S.random_field(p.shape, 6)).float()
    ref = O.residual_adjoint(oracle_params(p), widened(q32), widened(r32))
    prec = tgv.PRESETS["SP"]
    qb = torch.zeros(p.shape, dtype=torch.float32, device=DEV)
    tgv.ns_residual_adjoint(p, prec, q32.to(DEV), r32.to(DEV), qb,
                            work_for(p, prec, tgv.ns_residual_adjoint_workspace_bytes))
    scale = np.abs(ref).reshape(5, -1).max(1)
    err = np.abs(widened(qb) - ref).reshape(5, -1).max(1)
    say("  SP err / max|adjoint|", err / scale)
    assert np.all(err <= 2e-3 * scale)


@pytest.mark.parametrize("n", [(12, 16, 10), (5, 6, 7)])
def test_integrals_adjoint_matches_oracle(n):
    p = tgv.Params(n=n)
    q64 = S.random_state(n, 8, smooth=True)
    ref = O.integrals_adjoint(oracle_params(p), q64, 0.37)
    prec = tgv.PRESETS["DP"]
    qb = torch.zeros(p.shape, dtype=torch.float64, device=DEV)
    tgv.flow_integrals_adjoint(p, prec, torch.from_numpy(q64).to(DEV), 0.37, qb,
                               work_for(p, prec, tgv.flow_integrals_adjoint_workspace_bytes))
    scale = np.abs(ref).max()
    assert np.abs(qb.cpu().numpy() - ref).max() <= 1e-12 * scale


def test_rk_stage_adjoint_elementwise():
    p = tgv.Params(n=(7, 8, 9))
    prec = tgv.PRESETS["DP"]
    qb = torch.from_numpy(S.random_field(p.shape, 1)).to(DEV)
    z0 = S.random_field(p.shape, 2)
    for stage in (2, 1, 0):
        z = torch.from_numpy(z0).to(DEV)
        rb = torch.empty_like(z)
        tgv.rk_stage_adjoint(p, prec, stage, 0.01, qb, z, rb)
        bq = O.RK_B[stage] * qb.cpu().numpy()
        zz = z0 + bq
        scale = np.abs(z0) + np.abs(bq)  # the sum may cancel: bound on the operands
        assert np.all(np.abs(rb.cpu().numpy() - 0.01 * zz) <= 4e-16 * 0.01 * scale)
        assert np.all(np.abs(z.cpu().numpy() - O.RK_A[stage] * zz) <= 4e-16 * abs(O.RK_A[stage]) * scale)


@pytest.mark.parametrize("slots", [0, 1, 2, 5])
def test_trajectory_gradient_matches_oracle(slots):
    say("trajectory gradient slots", slots)
    n, dt, nsteps = (12, 12, 12), 0.01, 6
    p = tgv.Params(n=n)
    q0 = O.init(oracle_params(p))
    J_ref, g_ref = O.dissipation_grad(oracle_params(p), dt, nsteps, q0)
    runner = CheckpointedDissipation(p, tgv.PRESETS["DP"], dt, nsteps, slots=slots)
    q0d = torch.from_numpy(q0).to(DEV)
    J = runner.forward(q0d)
    g = runner.backward(q0d).cpu().numpy()
    assert abs(J - J_ref) <= 1e-13 * abs(J_ref)
    rel = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    say("  grad rel err", rel, "advances", runner.advances)
    assert rel <= 1e-11


def test_checkpointed_gradient_bitwise_equals_store_all():
    n, dt, nsteps = (10, 12, 8), 0.01, 9
    p = tgv.Params(n=n)
    q0 = torch.from_numpy(S.random_state(n, 3, smooth=True)).to(DEV)
    grads = []
    for slots in (1, 3, nsteps - 1):
        runner = CheckpointedDissipation(p, tgv.PRESETS["DP"], dt, nsteps, slots=slots)
        runner.forward(q0)
        grads.append(runner.backward(q0))
    assert torch.equal(grads[0], grads[2]) and torch.equal(grads[1], grads[2])


def test_autograd_velocity_gradient_matches_finite_differences():
    """dJ/du0 through torch autograd (state_from_velocity) and the revolve
    adjoint, against central differences with eps = 1e-6 along seeded
    Gaussian directions (unnormalised)."""
    n, dt, nsteps = (16, 16, 16), 0.02, 20
    p = tgv.Params(n=n)
    q0 = torch.from_numpy(O.init(oracle_params(p))).to(DEV)
    rho0 = q0[0].clone()
    u0 = (q0[1:4] / rho0).clone().requires_grad_(True)
    E = q0[4] - 0.5 * rho0 * (q0[1:4] / rho0).pow(2).sum(0)
    p0 = E * (p.gamma - 1.0)
    J = dissipation(state_from_velocity(u0, rho0, p0, p.gamma), p, tgv.PRESETS["DP"], dt, nsteps, slots=4)
    J.backward()
    g = u0.grad.detach()
    runner = CheckpointedDissipation(p, tgv.PRESETS["DP"], dt, nsteps, slots=4)
    eps = 1e-6
    for s in range(2):
        d = torch.from_numpy(S.directions(n, s)).to(DEV)
        with torch.no_grad():
            Jp = runner.forward(state_from_velocity(u0 + eps * d, rho0, p0, p.gamma))
            Jm = runner.forward(state_from_velocity(u0 - eps * d, rho0, p0, p.gamma))
        fd = (Jp - Jm) / (2 * eps)
        ad = float((g * d).sum())
        say("  FD", fd, "AD", ad)
        assert abs(fd - ad) <= 1e-6 * abs(ad)


@pytest.mark.parametrize("viscous", [1, 0])
def test_residual_adjoint_full_size_dot_product(viscous):
    """The benchmark's launch of ns_residual_adjoint (FP64, 512^3), checked by
    the adjoint identity <R_bar, J dQ> = <J^T R_bar, dQ>, which holds at any
    size: J dQ from central differences of the forward residual (itself
    checked against the oracle at this size on sampled points), eps = 1e-6
    (truncation and rounding each ~1e-10 relative here; a term missing from
    the viscous part alone would show at ~1e-4)."""
    n = 512
    say("adjoint dot product", n, "viscous", viscous)
    p = tgv.Params(n=(n, n, n), viscous=viscous)
    prec = tgv.PRESETS["DP"]
    gen = torch.Generator(device=DEV)
    gen.manual_seed(20250527 + viscous)
    draw = lambda: torch.randn(p.shape, generator=gen, dtype=torch.float64, device=DEV)
    scale = torch.tensor([1.0, 0.1, 0.1, 0.1, 1.0], dtype=torch.float64, device=DEV).view(5, 1, 1, 1)
    q = torch.empty(p.shape, dtype=torch.float64, device=DEV)
    tgv.tgv_init(p, q)
    q += 1e-3 * scale * draw()  # break the Taylor-Green symmetries
    dq = scale * draw()
    rbar = draw()
    eps = 1e-6
    r_p, r_m = torch.empty_like(q), torch.empty_like(q)
    tgv.ns_residual(p, prec, q + eps * dq, r_p)
    tgv.ns_residual(p, prec, q - eps * dq, r_m)
    r_p -= r_m
    lhs = float((r_p * rbar).sum()) / (2 * eps)
    del r_p, r_m
    qb = torch.zeros_like(q)
    tgv.ns_residual_adjoint(p, prec, q, rbar, qb, work_for(p, prec, tgv.ns_residual_adjoint_workspace_bytes))
    rhs = float((qb * dq).sum())
    say(f"  <R_bar, J dQ> = {lhs:.15e}  <J^T R_bar, dQ> = {rhs:.15e}  rel {abs(lhs - rhs) / abs(rhs):.2e}")
    assert abs(lhs - rhs) <= 1e-7 * abs(rhs)
