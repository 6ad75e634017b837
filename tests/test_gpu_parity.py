"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded
inputs.  FP64 bar: 1e-12 relative (to the term magnitude for the residual,
whose outputs are cancellations of much larger terms).  Reduced forms: the
rounding bound of the arithmetic and storage types."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import tgv_synth as S
from paper_2505_20911_amd import tgv
from paper_2505_20911_amd.solver import TGVSolver
from tgv_testutil import UNIT_ROUNDOFF, oracle_params, rounded, term_scale, widened

pytestmark = pytest.mark.gpu

DEV = "cuda"
GRIDS = [(16, 16, 16), (32, 32, 32), (24, 32, 40), (5, 6, 7), (70, 20, 37), (69, 20, 37), (128, 16, 64)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def state(kind, n, seed=0):
    if kind == "tgv":
        return O.init(O.Params(n=tuple(n)))
    if kind == "noise":
        return S.random_state(n, seed)
    return S.random_state(n, seed, smooth=True)


# ---------------------------------------------------------------- init
@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16, torch.bfloat16])
def test_init_matches_oracle(n, dtype):
    say("init", n, dtype)
    p = tgv.Params(n=n)
    q = torch.empty(p.shape, dtype=dtype, device=DEV)
    tgv.tgv_init(p, q)
    got = widened(q)
    ref = O.init(oracle_params(p))
    if dtype == torch.float64:
        assert np.all(np.abs(got - ref) <= 4e-16 * np.abs(ref).reshape(5, -1).max(1)[:, None, None, None])
    else:
        # correctly rounded FP64 values; sin/cos of two libraries may differ by
        # an FP64 ulp, which can move a value across a rounding boundary: allow
        # one unit of the storage precision.
        # Values near zero (sin of a multiple of pi) differ between the two
        # libraries in absolute terms: floor of 4 FP64 ulps of the field scale.
        u = UNIT_ROUNDOFF[dtype]
        floor = 4e-16 * np.abs(ref).reshape(5, -1).max(1)[:, None, None, None]
        assert np.all(np.abs(got - ref) <= 2 * u * np.abs(ref) + floor + 1e-300)
        exact = widened(rounded(ref, dtype)) if dtype != torch.bfloat16 else None
        if exact is not None:
            assert np.mean(got == exact) > 0.999


# ---------------------------------------------------------------- residual, FP64
@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("kind", ["tgv", "noise", "smooth"])
@pytest.mark.parametrize("viscous", [1, 0])
def test_residual_dp_matches_oracle(n, kind, viscous):
    say("residual DP", n, kind, viscous)
    p = tgv.Params(n=n, viscous=viscous)
    q64 = state(kind, n, seed=7)
    ref = O.residual(oracle_params(p), q64)
    q = torch.from_numpy(q64).to(DEV)
    r = torch.empty_like(q)
    tgv.ns_residual(p, tgv.PRESETS["DP"], q, r)
    got = widened(r)
    scale = term_scale(p.n, p.L, p.gamma, q64)
    err = np.abs(got - ref).reshape(5, -1).max(1)
    say("  max err / term scale", err / scale)
    assert np.all(err <= 1e-12 * scale), (err, scale)


# ---------------------------------------------------------------- residual, reduced forms
@pytest.mark.parametrize("form", ["SPDP", "SPDP_C64", "SP_DPC", "SP", "HPSP", "HPSP_BF16", "HP", "SPDP_WK", "HPSP_WK",
                                  "HPSP_RESWK", "HP_C16"])
@pytest.mark.parametrize("kind", ["tgv", "smooth"])
@pytest.mark.parametrize("n", [(24, 32, 16), (69, 20, 17)])  # odd nx: single-element plane loads
def test_residual_reduced_forms_within_rounding_bound(form, kind, n):
    """Q rounded to the storage type is the common input (the oracle sees it
    widened exactly); the GPU result may differ by the arithmetic type's
    rounding on the term scale plus one rounding of R to its storage type."""
    say("residual", form, kind, n)
    prec = tgv.PRESETS[form]
    p = tgv.Params(n=n)
    qs = rounded(state(kind, n, seed=3), prec.q)
    q64 = widened(qs)
    ref = O.residual(oracle_params(p), q64)
    r = torch.empty(p.shape, dtype=prec.r, device=DEV)
    tgv.ns_residual(p, prec, qs.to(DEV), r)
    got = widened(r)
    uc, ur = UNIT_ROUNDOFF[prec.compute], UNIT_ROUNDOFF[prec.r]
    scale = term_scale(p.n, p.L, p.gamma, q64)[:, None, None, None]
    tol = 64 * uc * scale + 2 * ur * np.abs(ref)
    bad = np.abs(got - ref) > tol
    say("  max err / (uc * scale)", (np.abs(got - ref) / (uc * scale)).reshape(5, -1).max(1))
    assert not bad.any()


def test_residual_uniform_state_is_exactly_zero():
    p = tgv.Params(n=(8, 10, 12))
    q = torch.empty(p.shape, dtype=torch.float64, device=DEV)
    rho, U, p0 = 1.3, (0.2, -0.4, 0.1), 50.0
    q[0] = rho
    for a in range(3):
        q[a + 1] = rho * U[a]
    q[4] = p0 / 0.4 + 0.5 * rho * sum(x * x for x in U)
    r = torch.full_like(q, 7.0)
    tgv.ns_residual(p, tgv.PRESETS["DP"], q, r)
    nz = (r != 0)
    if nz.any():
        idx = nz.nonzero()[:8].tolist()
        say("  nonzero:", int(nz.sum()), "max", float(r.abs().max()), "at", idx,
            "values", [float(r[tuple(i)]) for i in idx])
    assert not nz.any()


def test_residual_is_deterministic():
    p = tgv.Params(n=(24, 32, 40))
    q = torch.from_numpy(S.random_state(p.n, 9)).to(DEV)
    r1, r2 = torch.empty_like(q), torch.empty_like(q)
    tgv.ns_residual(p, tgv.PRESETS["DP"], q, r1)
    tgv.ns_residual(p, tgv.PRESETS["DP"], q, r2)
    assert torch.equal(r1, r2)


# ---------------------------------------------------------------- RK stage
@pytest.mark.parametrize("form", ["DP", "SPDP", "SP_DPC", "SP", "HPSP", "HPSP_BF16", "HP", "SPDP_WK", "HPSP_WK",
                                  "HPSP_RESWK", "HP_C16"])
@pytest.mark.parametrize("stage", [0, 1, 2])
def test_rk_stage_matches_oracle(form, stage):
    say("rk", form, stage)
    prec = tgv.PRESETS[form]
    p = tgv.Params(n=(9, 10, 11))  # 5N not a multiple of the vector width: exercises the tail
    rng = np.random.default_rng(stage)
    q = rounded(S.random_state(p.n, 1), prec.q)
    qt = rounded(rng.standard_normal(p.shape) * 0.01, prec.qt)
    r = rounded(rng.standard_normal(p.shape), prec.r)
    dt = 3.7e-3
    q64, qt64, r64 = widened(q), widened(qt), widened(r)
    if stage == 0:
        qt_in = torch.full_like(qt, float("nan"))  # stage 0 must not read the register
    else:
        qt_in = qt.clone()
    qd, qtd = q.to(DEV), qt_in.to(DEV)
    tgv.rk_stage(p, prec, stage, dt, qd, qtd, r.to(DEV))
    A, B = O.RK_A[stage], O.RK_B[stage]
    At = np.abs(A * qt64)  # |A qt| with the register before the stage
    q_in = q64.copy()
    O.rk_stage(stage, dt, q64, qt64, r64)  # updates q64, qt64 in place
    ua = 2.0 ** -53 if torch.float64 in (prec.q, prec.compute) else 2.0 ** -24
    uq, ut = UNIT_ROUNDOFF[prec.q], UNIT_ROUNDOFF[prec.qt]
    # half the smallest subnormal spacing of the storage types (FP16 register
    # values near zero round on an absolute grid)
    tiny_t = {torch.float16: 2.0 ** -25, torch.bfloat16: 2.0 ** -134}.get(prec.qt, 0.0)
    tiny_q = {torch.float16: 2.0 ** -25, torch.bfloat16: 2.0 ** -134}.get(prec.q, 0.0)
    got_t, got_q = widened(qtd), widened(qd)
    assert np.all(np.isfinite(got_t)) and np.all(np.isfinite(got_q))
    # register: two roundings in the arithmetic type on the operand scale, one
    # rounding to its storage type
    tol_t = 2 * ua * (At + dt * np.abs(r64)) + ut * np.abs(qt64) + tiny_t
    dt_err = np.abs(got_t - qt64)
    assert np.all(dt_err <= tol_t + 1e-300)
    # state: one fma on the scale |q| + |B t|, one rounding to storage, plus
    # the register difference carried through B
    tol_q = 2 * ua * (np.abs(q_in) + abs(B) * np.abs(qt64)) + uq * np.abs(q64) + abs(B) * dt_err + tiny_q
    assert np.all(np.abs(got_q - q64) <= tol_q + 1e-300)


# ---------------------------------------------------------------- fused residual + RK stage
@pytest.mark.parametrize("form", ["DP", "SPDP", "SPDP_C64", "SP_DPC", "SP", "HPSP", "HPSP_BF16", "HP", "SPDP_WK",
                                  "HPSP_WK", "HPSP_RESWK", "HP_C16"])
@pytest.mark.parametrize("n", [(24, 32, 40), (5, 6, 7), (64, 8, 70), (69, 20, 37), (130, 20, 9)])
def test_fused_stage_equals_residual_then_stage(form, n):
    """ns_residual_rk_stage is the same computation as ns_residual followed by
    rk_stage (R rounded to its storage type in both): bitwise equal."""
    say("fused", form, n)
    prec = tgv.PRESETS[form]
    p = tgv.Params(n=n)
    q0 = rounded(S.random_state(n, 2, smooth=True), prec.q).to(DEV)
    qt0 = rounded(np.random.default_rng(1).standard_normal(p.shape) * 1e-3, prec.qt).to(DEV)
    dt = 1e-3
    for stage in (0, 1, 2):
        qa, qta, r = q0.clone(), qt0.clone(), torch.empty(p.shape, dtype=prec.r, device=DEV)
        tgv.ns_residual(p, prec, qa, r)
        tgv.rk_stage(p, prec, stage, dt, qa, qta, r)
        qb, qtb = torch.empty_like(q0), qt0.clone()
        tgv.ns_residual_rk_stage(p, prec, stage, dt, q0, qb, qtb)
        assert torch.equal(qtb, qta), (stage, (qtb.double() - qta.double()).abs().max())
        assert torch.equal(qb, qa), (stage, (qb.double() - qa.double()).abs().max())


def test_fused_solver_trajectory_equals_split_solver():
    p = tgv.Params(n=(32, 32, 32))
    a = TGVSolver(p, tgv.PRESETS["DP"], fused=True)
    b = TGVSolver(p, tgv.PRESETS["DP"], fused=False)
    a.init()
    b.init()
    ha = a.run(7, 3.7e-3, every=1)
    hb = b.run(7, 3.7e-3, every=1)
    assert torch.equal(a.q, b.q) and torch.equal(ha, hb)


# ---------------------------------------------------------------- integrals
@pytest.mark.parametrize("n", GRIDS)
@pytest.mark.parametrize("kind", ["tgv", "noise"])
def test_integrals_match_oracle(n, kind):
    say("integrals", n, kind)
    p = tgv.Params(n=n)
    q64 = state(kind, n, seed=4)
    ref = O.integrals(oracle_params(p), q64)
    s = TGVSolver(p, tgv.PRESETS["DP"])
    s.q.copy_(torch.from_numpy(q64))
    got = s.integrals().cpu().numpy()
    scale = np.array([ref[0], ref[1], ref[2], 1.0, 1.0, 1.0, 1.0, ref[7]])
    assert np.all(np.abs(got - ref) <= 1e-13 * np.abs(scale)), (got - ref)


def test_integrals_of_taylor_green_state_closed_forms_at_256():
    """Properties that hold at any size: K0 = K_rho0 = 1/8 and the closed form
    eps^S(0) = (3/4) kprime(h)^2 / Re for the Taylor-Green state."""
    for n in (128, 256):
        p = tgv.Params(n=(n, n, n))
        s = TGVSolver(p, tgv.PRESETS["DP"])
        s.init()
        got = s.integrals().cpu().numpy()
        h = 2 * np.pi / n
        kp = (8 * np.sin(h) - np.sin(2 * h)) / (6 * h)
        assert abs(got[0] - 0.125) < 1e-14 and abs(got[1] - 0.125) < 1e-14
        assert abs(got[2] - 0.75 * kp * kp / 1600) < 1e-12 * got[2]
        assert abs(got[3] - 1.0) < 1e-14


# ---------------------------------------------------------------- end to end (32^3 DP, 50 steps)
def test_config_32cubed_trajectory_matches_oracle():
    say("trajectory 32^3 x 50 DP")
    n, dt, nsteps = (32, 32, 32), 3.7e-3, 50
    p = tgv.Params(n=n)
    q_ref, h_ref = O.run(oracle_params(p), dt, nsteps, every=1)
    s = TGVSolver(p, tgv.PRESETS["DP"])
    s.init()
    hist = s.run(nsteps, dt, every=1).cpu().numpy()
    q = s.q.cpu().numpy()
    q0 = O.init(oracle_params(p))
    for f in range(5):
        rel = np.linalg.norm(q[f] - q_ref[f]) / np.linalg.norm(q_ref[f])
        assert rel <= 1e-12, (f, rel)
        # the change over the run, which the mean of rho E hides
        dref = q_ref[f] - q0[f]
        if np.linalg.norm(dref) > 0:
            assert np.linalg.norm((q[f] - q0[f]) - dref) <= 1e-9 * np.linalg.norm(dref), f
    for m in (0, 1, 2):
        rel = np.abs(hist[:, m] - h_ref[:, m]) / np.abs(h_ref[:, m])
        assert rel.max() <= 1e-12, (m, rel.max())


# ---------------------------------------------------------------- full size, sampled
@pytest.mark.parametrize("n", [256, 512])
def test_residual_full_size_sampled(n):
    """At the benchmark's size the whole-field oracle is too slow: compare
    2000 sampled points (plus the 8 corners and edges of the periodic box)
    with the oracle's pointwise evaluation on the same input."""
    say("full size sampled", n)
    p = tgv.Params(n=(n, n, n))
    po = oracle_params(p)
    q64 = O.init(po)
    q64[1:4] *= 1.0 + 0.01 * np.cos(np.arange(n))[None, None, None, :]  # break the symmetry mildly
    rng = np.random.default_rng(n)
    idx = rng.choice(p.N, 2000, replace=False)
    edge = [0, n - 1, n * n - 1, n * n * (n - 1), p.N - 1, n // 2 + n * n * (n // 2)]
    idx = np.unique(np.concatenate([idx, edge])).astype(np.int64)
    ref = O.residual_at(po, q64, idx)
    q = torch.from_numpy(q64).to(DEV)
    del q64
    r = torch.empty_like(q)
    tgv.ns_residual(p, tgv.PRESETS["DP"], q, r)
    got = r.reshape(5, -1)[:, torch.from_numpy(idx).to(DEV)].T.cpu().numpy()
    # field magnitudes of the Taylor-Green state (read off a 16^3 copy), spacing of this grid
    scale = term_scale(p.n, p.L, p.gamma, O.init(oracle_params(tgv.Params(n=(16, 16, 16)))))
    assert np.all(np.abs(got - ref) <= 1e-12 * scale[None, :])


@pytest.mark.parametrize("n", [512, 1024])
def test_fused_stage_full_size_sampled(n):
    """The benchmark's launch: one fused residual + RK stage (stage 2 of 3,
    so both registers are read) in FP64 on the full grid, compared at 2000
    sampled points (plus corners and edges) with the oracle's pointwise
    residual combined by the stage formula in FP64."""
    say("fused full size sampled", n)
    p = tgv.Params(n=(n, n, n))
    po = oracle_params(p)
    q64 = O.init(po)
    q64[1:4] *= 1.0 + 0.01 * np.cos(np.arange(n))[None, None, None, :]
    rng = np.random.default_rng(n + 1)
    idx = rng.choice(p.N, 2000, replace=False)
    edge = [0, n - 1, n * n - 1, n * n * (n - 1), p.N - 1, n // 2 + n * n * (n // 2), n * n * (n - 2) + 3]
    idx = np.unique(np.concatenate([idx, edge])).astype(np.int64)
    R = O.residual_at(po, q64, idx)                   # (points, 5)
    q_s = q64.reshape(5, -1)[:, idx].T.copy()
    qt_s = 0.5 * q_s                                  # the Q~ register below is Q / 2, exact
    q = torch.from_numpy(q64).to(DEV)
    del q64
    qt = q * 0.5
    q_out = torch.empty_like(q)
    stage, dt = 1, 2.3125e-4
    tgv.ns_residual_rk_stage(p, tgv.PRESETS["DP"], stage, dt, q, q_out, qt)
    ti = torch.from_numpy(idx).to(DEV)
    got_qt = qt.reshape(5, -1)[:, ti].T.cpu().numpy()
    got_q = q_out.reshape(5, -1)[:, ti].T.cpu().numpy()
    del q, qt, q_out
    torch.cuda.empty_cache()
    A, B = O.RK_A[stage], O.RK_B[stage]
    ref_qt = A * qt_s + dt * R
    ref_q = q_s + B * ref_qt
    # field magnitudes of the Taylor-Green state (read off a 16^3 copy), spacing of this grid
    scale = term_scale(p.n, p.L, p.gamma, O.init(oracle_params(tgv.Params(n=(16, 16, 16)))))
    u = UNIT_ROUNDOFF[torch.float64]
    tol_qt = 4 * u * (np.abs(A * qt_s) + dt * np.abs(R)) + dt * 1e-12 * scale[None, :]
    tol_q = 4 * u * (np.abs(q_s) + np.abs(B * ref_qt)) + B * tol_qt
    assert np.all(np.abs(got_qt - ref_qt) <= tol_qt), np.max(np.abs(got_qt - ref_qt) / tol_qt)
    assert np.all(np.abs(got_q - ref_q) <= tol_q), np.max(np.abs(got_q - ref_q) / tol_q)


@pytest.mark.parametrize("form", ["SPDP", "SP", "HPSP", "HP"])
def test_fused_stage_full_size_sampled_reduced_forms(form):
    """The benchmark's launch for the reduced forms at 512^3: one fused stage
    (stage 2 of 3) on Q rounded to its storage type, compared at 2000 sampled
    points with the oracle's pointwise residual of the same (widened) Q, within
    the rounding bound of the arithmetic, R storage and register/state
    storage types."""
    say("fused full size sampled", form)
    n = 512
    prec = tgv.PRESETS[form]
    p = tgv.Params(n=(n, n, n))
    po = oracle_params(p)
    q64 = O.init(po)
    q64[1:4] *= 1.0 + 0.01 * np.cos(np.arange(n))[None, None, None, :]
    qs = rounded(q64, prec.q)
    del q64
    rng = np.random.default_rng(n + 2)
    idx = np.unique(np.concatenate([rng.choice(p.N, 2000, replace=False),
                                    [0, n - 1, n * n - 1, p.N - 1]])).astype(np.int64)
    qw = widened(qs)
    R = O.residual_at(po, qw, idx)
    scale = term_scale(p.n, p.L, p.gamma, qw)
    q_s = qw.reshape(5, -1)[:, idx].T.copy()
    del qw
    qt_s = 0.5 * q_s  # the register is Q / 2 (exact in every storage type here)
    q = qs.to(DEV)
    del qs
    qt = (q * 0.5).to(prec.qt)
    q_out = torch.empty_like(q)
    stage, dt = 1, 2.3125e-4
    tgv.ns_residual_rk_stage(p, prec, stage, dt, q, q_out, qt)
    ti = torch.from_numpy(idx).to(DEV)
    got_qt = widened(qt.reshape(5, -1)[:, ti].T)
    got_q = widened(q_out.reshape(5, -1)[:, ti].T)
    del q, qt, q_out
    torch.cuda.empty_cache()
    A, B = O.RK_A[stage], O.RK_B[stage]
    uc, ur = UNIT_ROUNDOFF[prec.compute], UNIT_ROUNDOFF[prec.r]
    ua = 2.0 ** -53 if torch.float64 in (prec.q, prec.compute) else 2.0 ** -24
    ut, uq = UNIT_ROUNDOFF[prec.qt], UNIT_ROUNDOFF[prec.q]
    tol_R = 64 * uc * scale[None, :] + 2 * ur * np.abs(R)
    ref_qt = A * qt_s + dt * R
    ref_q = q_s + B * ref_qt
    # half the smallest FP16 subnormal spacing: values near zero round on an absolute grid
    tiny_t = 2.0 ** -25 if prec.qt == torch.float16 else 0.0
    tiny_q = 2.0 ** -25 if prec.q == torch.float16 else 0.0
    tol_qt = dt * tol_R + 2 * ua * (np.abs(A * qt_s) + dt * np.abs(R)) + ut * np.abs(ref_qt) + tiny_t
    tol_q = B * tol_qt + 2 * ua * (np.abs(q_s) + abs(B) * np.abs(ref_qt)) + uq * np.abs(ref_q) + tiny_q
    say("  max err / tol", np.max(np.abs(got_qt - ref_qt) / tol_qt), np.max(np.abs(got_q - ref_q) / tol_q))
    assert np.all(np.abs(got_qt - ref_qt) <= tol_qt)
    assert np.all(np.abs(got_q - ref_q) <= tol_q)


def test_solver_on_a_side_stream_matches_default_stream():
    """Every entry point enqueues on the stream it is given: a run on a
    non-default stream (no implicit synchronisation with the default one) is
    bitwise equal to the same run on the default stream."""
    p = tgv.Params(n=(24, 32, 40))
    a = TGVSolver(p, tgv.PRESETS["DP"])
    a.init()
    ha = a.run(4, 3e-3, every=2)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        b = TGVSolver(p, tgv.PRESETS["DP"], stream=side.cuda_stream)
        b.init()
        hb = b.run(4, 3e-3, every=2)
    side.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(a.q, b.q) and torch.equal(ha, hb)
