"""GPU parity of the non-Blaisdell split forms of the convective term
(divergence, Feiereisen, Jameson, Kennedy-Gruber-Pirozzoli; Sec. 2.3.1 and the
inviscid comparison of Sec. 4.2) against the FP64 oracle: the same bars as the
Blaisdell form (FP64: 1e-12 of the term scale; half-single: the rounding bound
of its arithmetic and storage types) and the fused stage bitwise equal to the
residual followed by the stage."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import tgv_synth as S
from paper_2505_20911_amd import tgv
from tgv_testutil import UNIT_ROUNDOFF, oracle_params, rounded, term_scale, widened

pytestmark = pytest.mark.gpu
DEV = "cuda"
SPLITS = [(k, v) for k, v in tgv.SPLIT_FORMS.items() if v != 0]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def state(kind, n, seed):
    if kind == "tgv":
        return O.init(O.Params(n=tuple(n)))
    return S.random_state(n, seed, smooth=(kind == "smooth"))


@pytest.mark.parametrize("name,split", SPLITS)
@pytest.mark.parametrize("n", [(16, 16, 16), (70, 20, 37), (5, 6, 7)])
@pytest.mark.parametrize("kind", ["tgv", "noise", "smooth"])
@pytest.mark.parametrize("viscous", [1, 0])
def test_split_residual_dp_matches_oracle(name, split, n, kind, viscous):
    say("split", name, n, kind, viscous)
    p = tgv.Params(n=n, viscous=viscous, split=split)
    q64 = state(kind, n, 9)
    ref = O.residual(oracle_params(p), q64)
    q = torch.from_numpy(q64).to(DEV)
    r = torch.empty_like(q)
    tgv.ns_residual(p, tgv.PRESETS["DP"], q, r)
    scale = term_scale(p.n, p.L, p.gamma, q64)
    err = np.abs(widened(r) - ref).reshape(5, -1).max(1)
    say("  max err / term scale", err / scale)
    assert np.all(err <= 1e-12 * scale), (err, scale)


@pytest.mark.parametrize("name,split", SPLITS)
@pytest.mark.parametrize("kind", ["tgv", "smooth"])
def test_split_residual_hpsp_within_rounding_bound(name, split, kind):
    n = (24, 32, 16)
    prec = tgv.PRESETS["HPSP"]
    p = tgv.Params(n=n, split=split)
    qs = rounded(state(kind, n, 3), prec.q)
    q64 = widened(qs)
    ref = O.residual(oracle_params(p), q64)
    r = torch.empty(p.shape, dtype=prec.r, device=DEV)
    tgv.ns_residual(p, prec, qs.to(DEV), r)
    got = widened(r)
    uc, ur = UNIT_ROUNDOFF[prec.compute], UNIT_ROUNDOFF[prec.r]
    scale = term_scale(p.n, p.L, p.gamma, q64)[:, None, None, None]
    tol = 64 * uc * scale + 2 * ur * np.abs(ref)
    say("split HPSP", name, kind, (np.abs(got - ref) / (uc * scale)).reshape(5, -1).max(1))
    assert not (np.abs(got - ref) > tol).any()


@pytest.mark.parametrize("name,split", SPLITS)
@pytest.mark.parametrize("form", ["DP", "HPSP"])
def test_split_fused_stage_equals_residual_then_stage(name, split, form):
    prec = tgv.PRESETS[form]
    n = (70, 20, 37)
    p = tgv.Params(n=n, split=split)
    q0 = rounded(S.random_state(n, 2, smooth=True), prec.q).to(DEV)
    qt0 = rounded(np.random.default_rng(1).standard_normal(p.shape) * 1e-3, prec.qt).to(DEV)
    for stage in (0, 1, 2):
        qa, qta, r = q0.clone(), qt0.clone(), torch.empty(p.shape, dtype=prec.r, device=DEV)
        tgv.ns_residual(p, prec, qa, r)
        tgv.rk_stage(p, prec, stage, 4e-3, qa, qta, r)
        qb, qtb = torch.empty_like(q0), qt0.clone()
        tgv.ns_residual_rk_stage(p, prec, stage, 4e-3, q0, qb, qtb)
        assert torch.equal(qtb, qta) and torch.equal(qb, qa), (name, form, stage)


def test_split_forms_inviscid_trajectory_matches_oracle():
    """The robustness setting of the comparison (inviscid, M = 0.4, dt =
    0.004) on a small grid: 20 steps of every form in FP64 against the
    oracle's run, Q within 1e-12 relative L2 per field."""
    from paper_2505_20911_amd.solver import TGVSolver
    n = (16, 16, 16)
    for name, split in tgv.SPLIT_FORMS.items():
        p = tgv.Params(n=n, mach=0.4, viscous=0, split=split)
        q_ref, _ = O.run(oracle_params(p), 0.004, 20)
        s = TGVSolver(p, tgv.PRESETS["DP"])
        s.init()
        s.run(20, 0.004)
        q = s.q.cpu().numpy()
        for f in range(5):
            rel = np.linalg.norm(q[f] - q_ref[f]) / np.linalg.norm(q_ref[f])
            assert rel <= 1e-12, (name, f, rel)


@pytest.fixture(scope="module")
def tgv512():
    """Taylor-Green state at 512^3 with the symmetry mildly broken (FP64)."""
    n = 512
    q64 = O.init(oracle_params(tgv.Params(n=(n, n, n))))
    q64[1:4] *= 1.0 + 0.01 * np.cos(np.arange(n))[None, None, None, :]
    return q64


@pytest.mark.parametrize("name,split", SPLITS)
@pytest.mark.parametrize("form", ["DP", "HPSP"])
def test_split_fused_stage_full_size_sampled(name, split, form, tgv512):
    """The benchmark's split-form leg: one fused stage (stage 2 of 3) at 512^3
    in the DP and HPSP forms, compared at 2000 sampled points (plus corners)
    with the oracle's pointwise residual of the same split form combined by the
    stage formula: FP64 within 1e-12 of the term scale, HPSP within the
    rounding bound of its arithmetic and storage types."""
    say("split fused full size sampled", name, form)
    n = 512
    prec = tgv.PRESETS[form]
    p = tgv.Params(n=(n, n, n), split=split)
    po = oracle_params(p)
    qs = rounded(tgv512, prec.q)
    qw = widened(qs)
    rng = np.random.default_rng(n + 10 + split)
    idx = np.unique(np.concatenate([rng.choice(p.N, 2000, replace=False),
                                    [0, n - 1, n * n - 1, n * n * (n - 1), p.N - 1]])).astype(np.int64)
    R = O.residual_at(po, qw, idx)
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
    ref_qt = A * qt_s + dt * R
    ref_q = q_s + B * ref_qt
    # field magnitudes of the Taylor-Green state (read off a 16^3 copy), spacing of this grid
    scale = term_scale(p.n, p.L, p.gamma, O.init(oracle_params(tgv.Params(n=(16, 16, 16)))))
    if form == "DP":
        u = UNIT_ROUNDOFF[torch.float64]
        tol_qt = 4 * u * (np.abs(A * qt_s) + dt * np.abs(R)) + dt * 1e-12 * scale[None, :]
        tol_q = 4 * u * (np.abs(q_s) + np.abs(B * ref_qt)) + B * tol_qt
    else:
        uc, ur = UNIT_ROUNDOFF[prec.compute], UNIT_ROUNDOFF[prec.r]
        ua = 2.0 ** -24
        ut, uq = UNIT_ROUNDOFF[prec.qt], UNIT_ROUNDOFF[prec.q]
        tol_R = 64 * uc * scale[None, :] + 2 * ur * np.abs(R)
        tol_qt = dt * tol_R + 2 * ua * (np.abs(A * qt_s) + dt * np.abs(R)) + ut * np.abs(ref_qt)
        tol_q = B * tol_qt + 2 * ua * (np.abs(q_s) + abs(B) * np.abs(ref_qt)) + uq * np.abs(ref_q)
    say("  max err / tol", np.max(np.abs(got_qt - ref_qt) / tol_qt), np.max(np.abs(got_q - ref_q) / tol_q))
    assert np.all(np.abs(got_qt - ref_qt) <= tol_qt)
    assert np.all(np.abs(got_q - ref_q) <= tol_q)
