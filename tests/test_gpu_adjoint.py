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
from paper_2505_20911_amd.adjoint import (CheckpointedDissipation, dissipation, state_from_velocity,
                                          taylor_green_primitive)
from tgv_testutil import UNIT_ROUNDOFF, adjoint_term_scale, oracle_params, rounded, widened

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


# Grids on which the adjoint passes run a long plane march: the launch gives
# each block of 32 x 8 columns a chunk of up to 128 planes and halves the chunk
# (down to 4) until the grid holds at least 1024 blocks.  On 69 x 126 x 497 that
# is 16-plane chunks and 1536 blocks (a multiple of 8: XCD-contiguous block
# order on), ragged x (69 of 3 x 32 columns), y (126 of 16 x 8) and z
# (497 = 31 x 16 + 1: a one-plane last chunk), and 31 chunk seams along z, each
# with its 3-plane LDS ring restarted.  With odd nx the halo plane is loaded one
# point per lane; 70 x 126 x 497 is the same launch with even nx, where it is
# loaded in aligned x-pairs (the pairs crossing x = 0 of the periodic halo too).
FULL_LAUNCH_GRIDS = [(69, 126, 497), (70, 126, 497)]


def _plane_march(n):
    """Chunk height and block count of the adjoint launch on grid n (the rule
    the kernels' launcher applies)."""
    tx, ty, kz = -(-n[0] // 32), -(-n[1] // 8), 128
    while kz > 4 and tx * ty * -(-n[2] // kz) < 1024:
        kz //= 2
    return kz, tx * ty * -(-n[2] // kz)


@pytest.mark.parametrize("n", FULL_LAUNCH_GRIDS)
@pytest.mark.parametrize("viscous", [1, 0])
def test_residual_adjoint_dp_matches_oracle_in_the_full_launch(n, viscous):
    kz, blocks = _plane_march(n)
    assert kz == 16 and blocks % 8 == 0 and n[2] % kz != 0
    say("adjoint DP full launch", n, viscous, "kz", kz, "blocks", blocks)
    p = tgv.Params(n=n, viscous=viscous)
    q64 = S.random_state(n, 15, smooth=True)
    rbar = S.random_field(p.shape, 16)
    qb0 = S.random_field(p.shape, 17)
    ref = O.residual_adjoint(oracle_params(p), q64, rbar, qb0.copy())
    prec = tgv.PRESETS["DP"]
    qb = torch.from_numpy(qb0).to(DEV)
    tgv.ns_residual_adjoint(p, prec, torch.from_numpy(q64).to(DEV), torch.from_numpy(rbar).to(DEV), qb,
                            work_for(p, prec, tgv.ns_residual_adjoint_workspace_bytes))
    got = qb.cpu().numpy()
    scale = np.abs(ref - qb0).reshape(5, -1).max(1)
    err = np.abs(got - ref).reshape(5, -1).max(1)
    say("  err / max|adjoint|", err / scale)
    assert np.all(err <= 1e-12 * scale), err / scale


@pytest.mark.parametrize("n", [(12, 16, 10)] + FULL_LAUNCH_GRIDS)
@pytest.mark.parametrize("kind", ["tgv", "smooth"])
def test_residual_adjoint_sp_within_rounding(n, kind):
    """FP32 storage and arithmetic: the inputs rounded to FP32 are the common
    input (the oracle sees them widened exactly); the GPU result may differ by
    FP32 rounding on the adjoint's term scale (the same factor 64 of the unit
    roundoff as the forward residual's bound) plus one rounding of Q_bar."""
    say("adjoint SP", n, kind)
    p = tgv.Params(n=n)
    q64 = O.init(oracle_params(p)) if kind == "tgv" else S.random_state(n, 5, smooth=True)
    q32 = rounded(q64, torch.float32)
    r32 = rounded(S.random_field(p.shape, 6), torch.float32)
    ref = O.residual_adjoint(oracle_params(p), widened(q32), widened(r32))
    prec = tgv.PRESETS["SP"]
    qb = torch.zeros(p.shape, dtype=torch.float32, device=DEV)
    tgv.ns_residual_adjoint(p, prec, q32.to(DEV), r32.to(DEV), qb,
                            work_for(p, prec, tgv.ns_residual_adjoint_workspace_bytes))
    u = UNIT_ROUNDOFF[torch.float32]
    scale = adjoint_term_scale(p, widened(q32), widened(r32))
    err = np.abs(widened(qb) - ref)
    say("  SP err / (u * adjoint term scale)", (err / (u * scale)).reshape(5, -1).max(1),
        "max|adjoint| / term scale", np.abs(ref).max() / scale)
    assert np.all(err <= 64 * u * scale + 2 * u * np.abs(ref))


@pytest.mark.parametrize("n", [(12, 16, 10), (5, 6, 7)] + FULL_LAUNCH_GRIDS)
def test_integrals_adjoint_matches_oracle(n):
    say("eps^S adjoint DP", n)
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
    """dJ/du0 through the autograd function (the state map and its adjoint in
    the library) and the revolve adjoint, against central differences with
    eps = 1e-6 along seeded Gaussian directions (unnormalised), and against
    the oracle's store-all gradient carried to u0 by its chain rule."""
    n, dt, nsteps = (16, 16, 16), 0.02, 20
    p = tgv.Params(n=n)
    u0, rho0, p0 = taylor_green_primitive(p)
    uu = u0.clone().requires_grad_(True)
    J = dissipation(uu, rho0, p0, p, tgv.PRESETS["DP"], dt, nsteps, slots=4)
    J.backward()
    g = uu.grad.detach()
    po = oracle_params(p)
    uo, ro, pro = O.init_primitive(po)
    J_ref, gq_ref = O.dissipation_grad(po, dt, nsteps, O.velocity_ic_state(po, uo, ro, pro))
    g_ref = O.velocity_grad_from_state_grad(po, gq_ref, uo, ro)
    assert abs(float(J.detach()) - J_ref) <= 1e-13 * abs(J_ref)
    rel = float(np.linalg.norm(g.cpu().numpy() - g_ref) / np.linalg.norm(g_ref))
    say("  velocity gradient vs oracle, rel L2", rel)
    assert rel <= 1e-11
    runner = CheckpointedDissipation(p, tgv.PRESETS["DP"], dt, nsteps, slots=4)
    eps = 1e-6
    for s in range(2):
        d = torch.from_numpy(S.directions(n, s)).to(DEV)
        Jp = runner.forward(state_from_velocity(u0 + eps * d, rho0, p0, p))
        Jm = runner.forward(state_from_velocity(u0 - eps * d, rho0, p0, p))
        fd = (Jp - Jm) / (2 * eps)
        ad = float((g * d).sum())
        say("  FD", fd, "AD", ad)
        assert abs(fd - ad) <= 1e-6 * abs(ad)


@pytest.mark.parametrize("n", [(16, 16, 16), (69, 20, 37)])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_velocity_state_map_and_adjoint_match_oracle(n, dtype):
    """tgv_init_primitive, ns_state_from_velocity and its adjoint against the
    oracle's initial fields, velocity_ic_state and its chain rule (on the
    rounded inputs, widened exactly, for FP32)."""
    say("state map", n, dtype)
    p = tgv.Params(n=n)
    po = oracle_params(p)
    u, rho, pr = taylor_green_primitive(p, dtype)
    uo, ro, pro = O.init_primitive(po)
    u_ref = 1e-300 + np.abs(uo).max()
    if dtype == torch.float64:
        assert np.all(np.abs(widened(u) - uo) <= 4e-16 * u_ref)
        assert np.all(np.abs(widened(rho) - ro) <= 4e-16 * ro)
        assert np.all(np.abs(widened(pr) - pro) <= 4e-16 * pro)
    else:
        ur = UNIT_ROUNDOFF[dtype]
        assert np.all(np.abs(widened(u) - uo) <= ur * np.abs(uo) + 4e-16 * u_ref)
        assert np.all(np.abs(widened(rho) - ro) <= ur * ro)
        assert np.all(np.abs(widened(pr) - pro) <= ur * pro)
    # a perturbed velocity (not a symmetric field) through the state map
    d = rounded(0.1 * S.directions(n, 3), dtype).to(DEV)
    uu = u + d
    q = state_from_velocity(uu, rho, pr, p)
    q_ref = O.velocity_ic_state(po, widened(uu), widened(rho), widened(pr))
    uc = UNIT_ROUNDOFF[dtype]
    assert np.all(np.abs(widened(q) - q_ref) <= 4 * uc * np.abs(q_ref).reshape(5, -1).max(1)[:, None, None, None])
    qbar = rounded(S.random_field(p.shape, 9), dtype).to(DEV)
    ub = torch.empty_like(uu)
    tgv.ns_state_from_velocity_adjoint(p, uu, rho, qbar, ub)
    ub_ref = O.velocity_grad_from_state_grad(po, widened(qbar), widened(uu), widened(rho))
    scale = np.abs(widened(rho)).max() * (np.abs(widened(qbar)).max() * (1 + np.abs(widened(uu)).max()))
    assert np.all(np.abs(widened(ub) - ub_ref) <= 4 * uc * scale)


@pytest.mark.parametrize("rows", [1, 2, 3, 401, 1000])
def test_dissipation_trapezoid(rows):
    """J = dt sum_n w_n h[n, 2] with w_0 = w_{rows-1} = 1/2 (one row: 1/2),
    against an exactly rounded sum of the same terms."""
    import math
    h = S.random_field((rows, 8), rows) ** 2
    J = torch.empty(1, dtype=torch.float64, device=DEV)
    tgv.dissipation_trapezoid(torch.from_numpy(h).to(DEV), rows, 9.25e-4, J)
    w = [0.5 if k in (0, rows - 1) else 1.0 for k in range(rows)]
    ref = 9.25e-4 * math.fsum(wk * hk for wk, hk in zip(w, h[:, 2]))
    assert abs(float(J) - ref) <= 2 * rows * 2.0 ** -53 * abs(ref)


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
