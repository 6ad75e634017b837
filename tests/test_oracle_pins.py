"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

None of these checks re-types the oracle's own formulas: each compares it with
an independent fact -- a hand-evaluated fixture, a closed form (Fourier symbol,
discrete integral, RK stability polynomial, linearised acoustics), a symmetry,
a conservation law, a dense-matrix brute force, or convergence to the
continuous conservative-form Navier-Stokes equations evaluated spectrally.
"""
import math
import os

import numpy as np
import pytest

import oracle as O
from oracle import brute
import tgv_synth as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def P(n, **kw):
    if isinstance(n, int):
        n = (n, n, n)
    return O.Params(n=tuple(n), **kw)


def kprime(k, h):
    """Fourier symbol of the 4th-order central D1: D1 e^{ikx} = i kprime e^{ikx}."""
    return (8 * np.sin(k * h) - np.sin(2 * k * h)) / (6 * h)


def kpp2(k, h):
    """Minus the Fourier symbol of the 4th-order central D2."""
    return (30 - 32 * np.cos(k * h) + 2 * np.cos(2 * k * h)) / (12 * h * h)


# --------------------------------------------------------------------------
# Initial condition (Sec. 4.1)
# --------------------------------------------------------------------------

def test_ic_hand_evaluated_points():
    rows = np.loadtxt(os.path.join(GOLDEN, "tgv_ic_special_points.txt"))
    p = P(8)
    q = O.init(p)
    for row in rows:
        i, j, k = (int(v) for v in row[:3])
        np.testing.assert_allclose(q[:, k, j, i], row[3:], rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("n", [5, 8, 16, 32, (12, 20, 16)])
def test_ic_discrete_invariants(n):
    """K0 = K_rho0 = 1/8 exactly on any grid with n >= 5; <rho> = 1 and <p> = p0
    (the cosine terms average to zero); the discrete velocity divergence is
    (kprime(h_x) - kprime(h_y)) cos x cos y cos z (D1 sin = kprime cos), which
    vanishes on grids with h_x = h_y."""
    p = P(n)
    q = O.init(p)
    I = O.integrals(p, q)
    assert abs(I[0] - 0.125) < 1e-15
    assert abs(I[1] - 0.125) < 1e-15
    assert abs(I[3] - 1.0) < 1e-15
    gm2 = p.gamma * p.mach ** 2
    # <rho E> = <p>/(gamma-1) + K_rho = p0/(gamma-1) + 1/8, and the mean
    # momentum vanishes (every momentum component is odd under a reflection)
    E0 = 1 / gm2 / (p.gamma - 1) + 0.125
    assert abs(I[7] - E0) <= 4e-16 * E0
    assert np.all(np.abs(I[4:7]) <= 1e-16)
    rho, m, E = q[0], q[1:4], q[4]
    pr = (p.gamma - 1) * (E - 0.5 * (m ** 2).sum(0) / rho)
    assert abs(pr.mean() - 1 / gm2) < 1e-12
    u = m / rho
    div = sum(O.d1(p, u[a], a) for a in range(3))
    nx, ny, nz = p.n
    z, y, x = np.meshgrid(*(np.arange(m_) * 2 * np.pi / m_ for m_ in (nz, ny, nx)), indexing="ij")
    expect = (kprime(1, p.h(0)) - kprime(1, p.h(1))) * np.cos(x) * np.cos(y) * np.cos(z)
    assert np.abs(div - expect).max() < 1e-13


@pytest.mark.parametrize("n", [8, (12, 20, 16), 64])
def test_ic_pointwise_evaluator(n):
    """init_at (the pointwise initial state, used for sampled checks at sizes
    where the whole field is not formed) equals init element by element, and
    the hand-evaluated points of the golden fixture."""
    p = P(n)
    q = O.init(p).reshape(5, -1)
    idx = np.random.default_rng(5).choice(p.N, min(p.N, 4096), replace=False)
    got = O.init_at(p, idx)
    assert np.array_equal(got, q[:, idx].T)
    if n == 8:
        rows = np.loadtxt(os.path.join(GOLDEN, "tgv_ic_special_points.txt"))
        lin = [(int(r[2]) * 8 + int(r[1])) * 8 + int(r[0]) for r in rows]
        np.testing.assert_allclose(O.init_at(p, lin), rows[:, 3:], rtol=1e-14, atol=1e-14)


def test_ic_primitive_fields():
    """init_primitive (u, rho, p) at the hand-evaluated points of the golden
    fixture (velocity = momentum / rho there, p from rho = gamma M^2 p), and
    the state it gives through velocity_ic_state equals init."""
    p = P(8)
    u, rho, pr = O.init_primitive(p)
    rows = np.loadtxt(os.path.join(GOLDEN, "tgv_ic_special_points.txt"))
    for r in rows:
        i, j, k = int(r[0]), int(r[1]), int(r[2])
        np.testing.assert_allclose(rho[k, j, i], r[3], rtol=1e-15)
        np.testing.assert_allclose(u[:, k, j, i], r[4:7] / r[3], rtol=1e-15, atol=1e-16)
        np.testing.assert_allclose(pr[k, j, i], r[3] / (1.4 * 0.01), rtol=1e-15)
    for n in (8, (12, 20, 16)):
        p = P(n)
        u, rho, pr = O.init_primitive(p)
        np.testing.assert_allclose(O.velocity_ic_state(p, u, rho, pr), O.init(p), rtol=4e-16, atol=4e-16)


def test_velocity_state_chain_rule_by_complex_step():
    """velocity_grad_from_state_grad is the gradient of <q_bar, Q(u)> with
    respect to u for the map velocity_ic_state (density and pressure fixed):
    the complex-step derivative along a direction d equals <u_bar, d>."""
    p = P((6, 7, 5))
    u = S.random_field((3,) + p.shape[1:], 1) * 0.3
    rho = 1.0 + 0.1 * S.random_field(p.shape[1:], 2)
    pr = 70.0 + S.random_field(p.shape[1:], 3)
    qbar = S.random_field(p.shape, 4)
    ub = O.velocity_grad_from_state_grad(p, qbar, u, rho)
    for seed in (5, 6):
        d = S.random_field(u.shape, seed)
        h = 1e-30
        jd = (qbar * O.velocity_ic_state(p, u + 1j * h * d, rho, pr)).sum().imag / h
        assert abs(jd - (ub * d).sum()) <= 1e-13 * np.abs(ub * d).sum()


@pytest.mark.parametrize("n", [8, 16, 32])
def test_ic_reflection_symmetries(n):
    """u odd in x, v odd in y, w = 0, scalars even under each reflection x_d -> -x_d."""
    p = P(n)
    q = O.init(p)
    ref = lambda f, ax: np.roll(np.flip(f, axis=ax), 1, axis=ax)  # i -> (n - i) mod n
    for d, ax in ((0, 2), (1, 1), (2, 0)):
        for f in range(5):
            sign = -1.0 if f == d + 1 else 1.0
            np.testing.assert_allclose(ref(q[f], ax), sign * q[f], atol=1e-13)


@pytest.mark.parametrize("n", [16, 32, 128, 256])
def test_initial_dissipation_closed_form(n):
    """eps^S(0) = (3/4) kprime(1,h)^2 / Re exactly: every velocity factor is a
    single Fourier mode, so each discrete derivative is kprime times the
    conjugate mode and the grid means of sin^2, cos^2 are 1/2."""
    p = P((n, n, n)) if n <= 32 else None
    h = 2 * np.pi / n
    closed = 0.75 * kprime(1, h) ** 2 / 1600.0
    if p is not None:
        I = O.integrals(p, O.init(p))
        assert abs(I[2] - closed) / closed < 1e-14
    else:
        # printed reference values of the closed form at 128^3 / 256^3
        ref = {128: 4.6874981861e-4, 256: 4.6874998866e-4}[n]
        assert abs(closed - ref) / ref < 1e-10


# --------------------------------------------------------------------------
# Operators (Sec. 2.3.1: explicit 4th-order central differences)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("k", [1, 3, 5])
def test_operator_fourier_symbols(axis, k):
    n = (24, 20, 16)
    p = P(n)
    nx, ny, nz = n
    z, y, x = np.meshgrid(np.arange(nz) * 2 * np.pi / nz, np.arange(ny) * 2 * np.pi / ny,
                          np.arange(nx) * 2 * np.pi / nx, indexing="ij")
    X = (x, y, z)[axis]
    h = 2 * np.pi / n[axis]
    f = np.sin(k * X + 0.3) * (1.0 + 0.0 * x)
    np.testing.assert_allclose(O.d1(p, f, axis), kprime(k, h) * np.cos(k * X + 0.3), atol=1e-13)
    np.testing.assert_allclose(O.d2(p, f, axis), -kpp2(k, h) * f, atol=1e-12)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_operator_order_four(axis):
    errs1, errs2 = [], []
    for m in (16, 32, 64, 128):
        n = [8, 8, 8]
        n[axis] = m
        p = P(tuple(n))
        nx, ny, nz = n
        z, y, x = np.meshgrid(np.arange(nz) * 2 * np.pi / nz, np.arange(ny) * 2 * np.pi / ny,
                              np.arange(nx) * 2 * np.pi / nx, indexing="ij")
        X = (x, y, z)[axis]
        f = np.exp(np.sin(X))
        errs1.append(np.abs(O.d1(p, f, axis) - np.cos(X) * f).max())
        errs2.append(np.abs(O.d2(p, f, axis) - (np.cos(X) ** 2 - np.sin(X)) * f).max())
    for errs in (errs1, errs2):
        orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
        assert abs(orders[-1] - 4.0) < 0.05, orders


# --------------------------------------------------------------------------
# Full residual
# --------------------------------------------------------------------------

def spectral_residual(rho, u, p, gamma, mach, re, pr, viscous=True):
    """The continuous compressible Navier-Stokes right-hand side in plain
    conservative form, with exact (FFT) derivatives on a periodic grid of the
    analytic fields rho, u (3), p shaped (nz, ny, nx) on [0, 2 pi)^3.  Constant
    mu = 1, Stokes stress, Fourier heat flux, p = rho T / (gamma M^2)."""
    nz, ny, nx = rho.shape
    k = [np.fft.fftfreq(m, 1.0 / m) for m in (nx, ny, nz)]

    def D(f, d):
        ax = 2 - d
        shape = [1, 1, 1]
        shape[ax] = f.shape[ax]
        kk = k[d].reshape(shape)
        return np.real(np.fft.ifft(1j * kk * np.fft.fft(f, axis=ax), axis=ax))

    m = [rho * u[a] for a in range(3)]
    E = p / (gamma - 1) + 0.5 * rho * sum(u[a] ** 2 for a in range(3))
    R = np.zeros((5,) + rho.shape)
    R[0] = -sum(D(m[j], j) for j in range(3))
    for i in range(3):
        R[i + 1] = -sum(D(m[i] * u[j] + (p if i == j else 0.0), j) for j in range(3))
    R[4] = -sum(D((E + p) * u[j], j) for j in range(3))
    if viscous:
        G = [[D(u[i], j) for j in range(3)] for i in range(3)]
        div = G[0][0] + G[1][1] + G[2][2]
        tau = [[(G[i][j] + G[j][i] - (2.0 / 3.0 if i == j else 0.0) * div) / re
                for j in range(3)] for i in range(3)]
        T = gamma * mach ** 2 * p / rho
        kappa = 1.0 / ((gamma - 1) * mach ** 2 * pr * re)
        for i in range(3):
            R[i + 1] += sum(D(tau[i][j], j) for j in range(3))
        R[4] += sum(D(sum(u[i] * tau[i][j] for i in range(3)), j) for j in range(3))
        R[4] += sum(D(kappa * D(T, j), j) for j in range(3))
    return R


def analytic_state(n):
    z, y, x = np.meshgrid(*(np.arange(m) * 2 * np.pi / m for m in (n, n, n)), indexing="ij")
    rho = 1.0 + 0.2 * np.sin(x) * np.cos(y) * np.sin(z + 0.3)
    u = [0.5 * np.sin(x + 0.1) * np.cos(2 * y) + 0.1,
         0.4 * np.cos(x) * np.sin(y + 0.7) * np.cos(z),
         0.3 * np.sin(z) * np.cos(x + y) - 0.05]
    return x, y, z, rho, u


@pytest.mark.parametrize("viscous", [1, 0])
def test_residual_converges_to_continuous_equations(viscous):
    """The discrete residual (any split form, D2 vs D1 D1) must converge at 4th
    order to the continuous conservative-form equations.  Low Re and M = 0.5
    make the viscous, heat-flux and pressure terms O(1) so that a dropped term,
    wrong sign or wrong coefficient anywhere shows up as a non-converging error."""
    gamma, mach, re, pr = 1.4, 0.5, 10.0, 0.71
    nf = 128
    _, _, _, rho_f, u_f = analytic_state(nf)
    z, y, x = np.meshgrid(*(np.arange(m) * 2 * np.pi / m for m in (nf, nf, nf)), indexing="ij")
    p_f = (1.0 / (gamma * mach ** 2)) * (1.0 + 0.1 * np.cos(x + z) + 0.05 * np.sin(2 * y))
    Rref_f = spectral_residual(rho_f, u_f, p_f, gamma, mach, re, pr, bool(viscous))
    errs = []
    for n in (16, 32, 64):
        s = nf // n
        rho = rho_f[::s, ::s, ::s]
        u = [uu[::s, ::s, ::s] for uu in u_f]
        pp = p_f[::s, ::s, ::s]
        q = np.empty((5, n, n, n))
        q[0] = rho
        for a in range(3):
            q[a + 1] = rho * u[a]
        q[4] = pp / (gamma - 1) + 0.5 * rho * sum(uu ** 2 for uu in u)
        prm = P(n, gamma=gamma, mach=mach, re=re, pr=pr, viscous=viscous)
        R = O.residual(prm, q)
        Rref = Rref_f[:, ::s, ::s, ::s]
        errs.append(np.abs(R - Rref).reshape(5, -1).max(axis=1))
    errs = np.array(errs)
    for f in range(5):
        order = math.log2(errs[1, f] / errs[2, f])
        assert 3.7 < order < 4.4, (f, errs[:, f])
        assert errs[0, f] > errs[1, f] > errs[2, f]


def term_scale(p, q):
    """Magnitude of the individual flux-derivative terms of each residual
    component, (max|q_f| (1 + max|u|) + max|p|) / h_min: rounding errors of
    any evaluation order are relative to this, not to R, which at the TGV
    state is a cancellation of terms of size ~|rho E| / h down to O(1)."""
    rho, m, E = q[0], q[1:4], q[4]
    umax = np.abs(m / rho).max()
    pmax = np.abs((p.gamma - 1) * (E - 0.5 * (m * m).sum(0) / rho)).max()
    h = min(p.h(d) for d in range(3))
    return np.array([(np.abs(q[f]).max() * (1 + umax) + pmax) / h for f in range(5)])


def test_residual_matches_dense_brute_force_tgv_and_random():
    p = P(16)
    for q in (O.init(p), S.random_state(p.n, 11), S.random_state(p.n, 12, smooth=True)):
        for visc in (1, 0):
            p.viscous = visc
            r = O.residual(p, q)
            rb = brute.residual(q, p.n, p.L, p.gamma, p.mach, p.re, p.pr, bool(visc))
            err = np.abs(r - rb).reshape(5, -1).max(axis=1)
            assert np.all(err <= 1e-15 * term_scale(p, q)), (err, term_scale(p, q))


# --------------------------------------------------------------------------
# Split forms of the convective term (Sec. 2.3.1; inviscid comparison, Sec. 4.2)
# --------------------------------------------------------------------------

SPLITS = list(O.SPLIT_FORMS.items())


@pytest.mark.parametrize("name,split", SPLITS)
def test_split_form_matches_dense_brute_force(name, split):
    """The brute force builds each form from its pairing of the factors
    rho, u_j, phi (and KGP from its identity with the three pairings; Kok and
    KEEP from their two-point fluxes), not from the oracle's term list."""
    p = P((12, 10, 8), split=split)
    for q in (O.init(p), S.random_state(p.n, 31, smooth=True), S.random_state(p.n, 32)):
        for visc in (1, 0):
            p.viscous = visc
            r = O.residual(p, q)
            rb = brute.residual(q, p.n, p.L, p.gamma, p.mach, p.re, p.pr, bool(visc), name)
            err = np.abs(r - rb).reshape(5, -1).max(axis=1)
            assert np.all(err <= 1e-15 * term_scale(p, q)), (name, err)


@pytest.mark.parametrize("name,split", SPLITS)
def test_split_form_matches_two_point_flux_form(name, split):
    """Every split form written as the conservative difference of interface
    fluxes assembled from its symmetric two-point flux (Kok 2009; Kuya, Totani
    and Kawai 2018: {rho phi}{u}, {rho u}{phi}, {rho}{u}{phi}, ..., and for Kok
    and KEEP the internal-plus-kinetic energy flux with u_a(left) u_a(right)/2
    and the pressure flux (p_L u_R + p_R u_L)/2).  The oracle codes product-rule
    expansions instead; the two agree only if each expansion is the exact
    algebraic image of its flux."""
    p = P((12, 10, 8), split=split)
    for q in (O.init(p), S.random_state(p.n, 33, smooth=True), S.random_state(p.n, 34)):
        for visc in (1, 0):
            p.viscous = visc
            r = O.residual(p, q)
            rb = brute.residual(q, p.n, p.L, p.gamma, p.mach, p.re, p.pr, bool(visc), name, flux_form=True)
            err = np.abs(r - rb).reshape(5, -1).max(axis=1)
            assert np.all(err <= 4e-15 * term_scale(p, q)), (name, err / term_scale(p, q))


@pytest.mark.parametrize("name,split", SPLITS)
def test_kinetic_energy_preservation(name, split):
    """Semi-discrete kinetic energy budget of the inviscid residual:
    sum_i [u_a R_{m_a} - |u|^2 R_rho / 2] = sum_i p D_a u_a holds exactly (the
    convective terms neither create nor destroy kinetic energy; only the
    pressure-dilatation work remains) for the forms built on the (rho u) x u_a
    or rho x u x u_a pairings with a consistent mass flux -- Feiereisen, KGP,
    Kok and KEEP -- and fails, by far more than rounding, for the others."""
    p = P((12, 16, 10), viscous=0, split=split)
    q = S.random_state(p.n, 51)
    r = O.residual(p, q)
    ops = brute.Ops(p.n, p.L)
    rho = q[0]
    u = [q[a + 1] / rho for a in range(3)]
    pr = (p.gamma - 1) * (q[4] - 0.5 * sum(q[a + 1] * u[a] for a in range(3)))
    ke_rate = sum(u[a] * r[a + 1] for a in range(3)) - 0.5 * sum(uu ** 2 for uu in u) * r[0]
    work = pr * sum(ops.d1(u[a], a) for a in range(3))
    scale = np.abs(sum(u[a] * r[a + 1] for a in range(3))).sum() + np.abs(work).sum()
    gap = abs(ke_rate.sum() - work.sum()) / scale
    if name in ("feiereisen", "kgp", "kok", "keep"):
        assert gap <= 1e-15, (name, gap)
    else:
        assert gap >= 1e-8, (name, gap)


@pytest.mark.parametrize("name,split", SPLITS)
def test_split_form_converges_to_continuous_equations(name, split):
    """Every split form is a consistent discretisation of the same equations:
    4th-order convergence to the spectral conservative-form right-hand side
    (inviscid, M = 0.5 so pressure and convection are both O(1))."""
    gamma, mach = 1.4, 0.5
    nf = 128
    _, _, _, rho_f, u_f = analytic_state(nf)
    z, y, x = np.meshgrid(*(np.arange(m) * 2 * np.pi / m for m in (nf, nf, nf)), indexing="ij")
    p_f = (1.0 / (gamma * mach ** 2)) * (1.0 + 0.1 * np.cos(x + z) + 0.05 * np.sin(2 * y))
    Rref_f = spectral_residual(rho_f, u_f, p_f, gamma, mach, 10.0, 0.71, False)
    errs = []
    for n in (16, 32, 64):
        s = nf // n
        rho, u, pp = rho_f[::s, ::s, ::s], [uu[::s, ::s, ::s] for uu in u_f], p_f[::s, ::s, ::s]
        q = np.empty((5, n, n, n))
        q[0] = rho
        for a in range(3):
            q[a + 1] = rho * u[a]
        q[4] = pp / (gamma - 1) + 0.5 * rho * sum(uu ** 2 for uu in u)
        R = O.residual(P(n, gamma=gamma, mach=mach, viscous=0, split=split), q)
        errs.append(np.abs(R - Rref_f[:, ::s, ::s, ::s]).reshape(5, -1).max(axis=1))
    errs = np.array(errs)
    for f in range(5):
        order = math.log2(errs[1, f] / errs[2, f])
        assert 3.7 < order < 4.4, (name, f, errs[:, f])


@pytest.mark.parametrize("name,split", SPLITS)
def test_split_form_conserves_and_vanishes_on_uniform_states(name, split):
    """D1 is skew and its columns sum to zero, so every product-rule pair
    (a D b + b D a) and every divergence sums to zero over the periodic grid:
    mass, momentum and (inviscid) total energy are conserved by every form.
    A uniform state has zero residual in every form."""
    p = P((12, 16, 10), viscous=0, split=split)
    q = S.random_state(p.n, 21)
    r = O.residual(p, q).reshape(5, -1)
    for f in range(5):
        assert abs(r[f].sum()) < 1e-13 * np.abs(r[f]).sum(), (name, f)
    qu = np.empty(p.shape)
    qu[0] = 1.3
    for a, U in enumerate((0.2, -0.4, 0.1)):
        qu[a + 1] = 1.3 * U
    qu[4] = 50.0 / 0.4 + 0.5 * 1.3 * 0.21
    h = min(p.h(d) for d in range(3))
    assert np.abs(O.residual(p, qu)).max() < 1e-14 * np.abs(qu).max() / h ** 2


def test_split_forms_relations():
    """Exact relations between the forms: for phi = 1 (continuity) Feiereisen
    is the divergence form and Jameson and KGP are Blaisdell; and the cubic
    KGP form is (Blaisdell + Feiereisen + Jameson)/2 - divergence/2 for every
    component (the pressure and viscous terms, common to all, cancel)."""
    q = S.random_state((12, 10, 8), 41, smooth=True)
    R = {name: O.residual(P((12, 10, 8), split=k), q) for name, k in SPLITS}
    sc = term_scale(P((12, 10, 8)), q)
    close = lambda a, b, f: np.abs(a - b).max() <= 1e-14 * sc[f]
    assert close(R["feiereisen"][0], R["divergence"][0], 0)
    assert close(R["jameson"][0], R["blaisdell"][0], 0)
    assert close(R["kgp"][0], R["blaisdell"][0], 0)
    comb = 0.5 * (R["blaisdell"] + R["feiereisen"] + R["jameson"]) - 0.5 * R["divergence"]
    for f in range(5):
        assert close(R["kgp"][f], comb[f], f), f
    # Kok shares Feiereisen's mass and momentum terms, KEEP those of KGP; their
    # energy terms differ (internal + kinetic energy, split pressure work)
    for f in range(4):
        assert close(R["kok"][f], R["feiereisen"][f], f), f
        assert close(R["keep"][f], R["kgp"][f], f), f
    for a, b in (("kok", "feiereisen"), ("keep", "kgp"), ("kok", "keep")):
        assert np.abs(R[a][4] - R[b][4]).max() > 1e-5 * np.abs(R[b][4]).max(), (a, b)
    # and the forms do differ where phi varies (by their truncation errors)
    for a, b in (("feiereisen", "blaisdell"), ("jameson", "blaisdell"), ("divergence", "kgp")):
        assert np.abs(R[a][1] - R[b][1]).max() > 1e-4 * np.abs(R[b][1]).max(), (a, b)


@pytest.mark.parametrize("split", sorted(O.SPLIT_FORMS.values()))
def test_residual_pointwise_matches_whole_field(split):
    """The pointwise evaluator (used for sampled checks on full-size grids) is a
    second, independent transcription of the residual: every split form agrees
    with the whole-field oracle, which is pinned by the tests above."""
    p = P((12, 16, 20), split=split)
    q = S.random_state(p.n, 5)
    r = O.residual(p, q)
    idx = np.random.default_rng(0).choice(p.N, 300, replace=False)
    ra = O.residual_at(p, q, idx)
    scale = np.abs(r).max()
    np.testing.assert_allclose(ra, r.reshape(5, -1)[:, idx].T, atol=1e-14 * scale)


@pytest.mark.parametrize("visc", [1, 0])
def test_uniform_state_has_zero_residual(visc):
    p = P((8, 10, 12), viscous=visc)
    q = np.empty(p.shape)
    rho, U, p0 = 1.3, (0.2, -0.4, 0.1), 50.0
    q[0] = rho
    for a in range(3):
        q[a + 1] = rho * U[a]
    q[4] = p0 / 0.4 + 0.5 * rho * sum(x * x for x in U)
    r = O.residual(p, q)
    h = min(p.h(d) for d in range(3))
    assert np.abs(r).max() < 1e-14 * np.abs(q).max() / h ** 2


def test_conservation_of_mass_momentum_energy():
    """Column sums of D1, D2 and D1 D1 vanish and D1 is skew on the periodic
    grid, so the split convective forms, the pressure gradient and the viscous
    momentum terms sum to zero over the grid.  The total energy sums to zero
    only without viscosity (the product-rule viscous work with D2 != D1 D1 is
    not a discrete divergence)."""
    p = P((12, 16, 10))
    q = S.random_state(p.n, 21)
    for visc in (1, 0):
        p.viscous = visc
        r = O.residual(p, q).reshape(5, -1)
        for f in range(5):
            if f == 4 and visc:
                continue
            tot = r[f].sum()
            assert abs(tot) < 1e-13 * np.abs(r[f]).sum(), (f, tot)
    p.viscous = 1
    r = O.residual(p, q).reshape(5, -1)
    assert abs(r[4].sum()) > 1e-8 * np.abs(r[4]).sum()


def test_shift_equivariance_bitwise():
    p = P((12, 16, 10))
    q = S.random_state(p.n, 31)
    r = O.residual(p, q)
    sh = (3, -5, 2)  # (z, y, x) shifts in array axes
    qs = np.roll(q, sh, axis=(1, 2, 3))
    rs = O.residual(p, qs)
    assert np.array_equal(rs, np.roll(r, sh, axis=(1, 2, 3)))


def reflect(q, d):
    """x_d -> -x_d on the grid (i -> (n - i) mod n), flipping momentum d."""
    ax = 3 - d
    out = np.roll(np.flip(q, axis=ax), 1, axis=ax).copy()
    out[d + 1] *= -1
    return out


def rotate_z(q):
    """Rotation by +90 deg about z: F'(x, y) = F(y, -x); m'_x = -m_y, m'_y = m_x
    taken at the same source point."""
    nz, ny, nx = q.shape[1:]
    assert nx == ny
    i = np.arange(nx)
    j = np.arange(ny)
    J, I = np.meshgrid(j, i, indexing="ij")  # target (j, i)
    src_i = J  # source x index = target y index
    src_j = (-I) % nx  # source y index = -target x index
    out = q[:, :, src_j, src_i].copy()
    mx, my = out[1].copy(), out[2].copy()
    out[1] = -my
    out[2] = mx
    return out


def test_reflection_and_rotation_equivariance():
    p = P((12, 12, 10))
    q = S.random_state(p.n, 41)
    r = O.residual(p, q)
    scale = np.abs(r).reshape(5, -1).max(axis=1)[:, None, None, None]
    for d in range(3):
        assert np.all(np.abs(O.residual(p, reflect(q, d)) - reflect(r, d)) <= 1e-13 * scale)
    assert np.all(np.abs(O.residual(p, rotate_z(q)) - rotate_z(r)) <= 1e-13 * scale)
    # the rotation is not a symmetry of the field itself (the check is not vacuous)
    assert np.abs(rotate_z(q) - q).max() > 0.1


# --------------------------------------------------------------------------
# Time integration (Sec. 3.1 two-register RK update)
# --------------------------------------------------------------------------

def rk_poly(z):
    return 1 + z + z * z / 2 + z ** 3 / 6


def test_rk_scalar_amplification():
    """For y' = lam y one step of any 3-stage 3rd-order scheme multiplies y by
    P(lam dt) = 1 + z + z^2/2 + z^3/6."""
    lam = np.array([-1.0, -0.3, 0.5, -2.0, -0.05])
    dt = 0.37
    q = np.ones(5)
    qt = np.full(5, np.nan)  # stage 0 must not read the register
    r = np.empty(5)
    for s in range(3):
        r[:] = lam * q
        O.rk_stage(s, dt, q, qt, r)
    np.testing.assert_allclose(q, rk_poly(lam * dt), rtol=1e-15)


def test_rk_third_order_on_nonlinear_ode():
    """y' = -y^2, y(0) = 1, exact y = 1/(1 + t): global error falls by 8 per halving."""
    errs = []
    for nsteps in (20, 40, 80, 160):
        dt = 1.0 / nsteps
        q = np.ones(1)
        qt = np.zeros(1)
        r = np.empty(1)
        for _ in range(nsteps):
            for s in range(3):
                r[:] = -q * q
                O.rk_stage(s, dt, q, qt, r)
        errs.append(abs(q[0] - 0.5))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert abs(orders[-1] - 3.0) < 0.05, orders


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_inviscid_entropy_wave_fully_discrete(axis):
    """rho = 1 + eps sin(x_d), uniform velocity U along x_d and uniform p: the
    split convective terms reduce to linear advection of every conserved
    field, so each step multiplies the Fourier mode by P(-i U kprime dt)."""
    n = [8, 8, 8]
    n[axis] = 24
    p = P(tuple(n), viscous=0)
    nx, ny, nz = n
    z, y, x = np.meshgrid(*(np.arange(m) * 2 * np.pi / m for m in (nz, ny, nx)), indexing="ij")
    X = (x, y, z)[axis]
    eps, U, p0 = 0.1, 1.0, 1 / (1.4 * 0.01)
    q = np.zeros(p.shape)
    q[0] = 1 + eps * np.sin(X)
    q[axis + 1] = U * q[0]
    q[4] = p0 / 0.4 + 0.5 * U * U * q[0]
    dt, nsteps = 0.02, 40
    qn, _ = O.run(p, dt, nsteps, q)
    h = 2 * np.pi / n[axis]
    G = rk_poly(-1j * U * kprime(1, h) * dt) ** nsteps
    expect = 1 + eps * np.imag(G * np.exp(1j * X))
    np.testing.assert_allclose(qn[0], expect, atol=1e-13)


@pytest.mark.parametrize("a,d", [(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)])
def test_viscous_shear_wave_fully_discrete(a, d):
    """m_a = eps sin(x_d), d != a, rho = 1, uniform p: convection vanishes, the
    pressure and density respond only at O(eps^2), so the mode decays with
    P(-dt kpp2 / Re) per step -- the D2 symbol, not the D1 D1 one."""
    n = [8, 8, 8]
    n[d] = 16
    p = P(tuple(n))
    nx, ny, nz = n
    z, y, x = np.meshgrid(*(np.arange(m) * 2 * np.pi / m for m in (nz, ny, nx)), indexing="ij")
    X = (x, y, z)[d]
    eps, p0 = 1e-8, 1 / (1.4 * 0.01)
    q = np.zeros(p.shape)
    q[0] = 1.0
    q[a + 1] = eps * np.sin(X)
    q[4] = p0 / 0.4 + 0.5 * q[a + 1] ** 2
    dt, nsteps = 0.05, 30
    qn, _ = O.run(p, dt, nsteps, q)
    h = 2 * np.pi / n[d]
    g = rk_poly(-dt * kpp2(1, h) / p.re) ** nsteps
    np.testing.assert_allclose(qn[a + 1], g * eps * np.sin(X), atol=1e-12 * eps)
    # and the D1 D1 symbol would have been visibly different
    g_alt = rk_poly(-dt * kprime(1, h) ** 2 / p.re) ** nsteps
    assert abs(g - g_alt) > 1e-6


def linearised_symbol(k, h, d, rho0, U, p0, gamma, mach, re, pr, viscous):
    """5x5 matrix A with R'(mode e^{i k x_d}) = A delta for the perturbation
    (rho', m', rhoE') of a uniform state, derived from the linearised
    Navier-Stokes terms with the discrete symbols of D1 (i kprime) and D2 (-kpp2)."""
    s1 = 1j * kprime(k, h)
    s2 = -kpp2(k, h)
    U = np.asarray(U, float)
    E0 = p0 / (gamma - 1) + 0.5 * rho0 * U @ U
    q0 = np.array([rho0, rho0 * U[0], rho0 * U[1], rho0 * U[2], E0])
    Mu = np.zeros((3, 5))  # u' = (m' - U rho') / rho0
    for a in range(3):
        Mu[a, 0] = -U[a] / rho0
        Mu[a, a + 1] = 1.0 / rho0
    Mp = (gamma - 1) * np.array([0.5 * U @ U, -U[0], -U[1], -U[2], 1.0])
    gm2 = gamma * mach ** 2
    MT = gm2 * (Mp / rho0 - p0 / rho0 ** 2 * np.eye(5)[0])
    A = np.zeros((5, 5), complex)
    for f in range(5):  # convection
        A[f] -= s1 * (U[d] * np.eye(5)[f] + q0[f] * Mu[d])
    A[d + 1] -= s1 * Mp  # pressure
    A[4] -= s1 * (U[d] * Mp + p0 * Mu[d])
    if viscous:
        kap = 1.0 / ((gamma - 1) * mach ** 2 * pr * re)
        Vm = np.zeros((3, 5), complex)
        for a in range(3):
            Vm[a] = s2 * Mu[a] / re + (s2 * Mu[d] / (3 * re) if a == d else 0)
            A[a + 1] += Vm[a]
        A[4] += sum(U[a] * Vm[a] for a in range(3)) + kap * s2 * MT
    return A


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("viscous", [1, 0])
def test_linearised_dynamics_by_complex_step(d, viscous):
    """Complex step (h = 1e-20) of n full RK3 steps about a uniform moving
    state equals P(dt A)^n applied to the perturbation's Fourier amplitude,
    with A the linearised-equations symbol: pins the acoustic coupling, the
    equation of state, advection, 1/Re with the 4/3 longitudinal factor,
    the heat-flux coefficient and the RK update together."""
    gamma, mach, re, pr = 1.4, 0.3, 50.0, 0.71
    n = [6, 6, 6]
    n[d] = 16
    p = P(tuple(n), gamma=gamma, mach=mach, re=re, pr=pr, viscous=viscous)
    rho0, U, p0 = 1.1, (0.3, -0.2, 0.25), 1 / (gamma * mach ** 2)
    nx, ny, nz = n
    z, y, x = np.meshgrid(*(np.arange(m) * 2 * np.pi / m for m in (nz, ny, nx)), indexing="ij")
    X = (x, y, z)[d]
    k = 2
    vhat = np.array([0.3 + 0.1j, -0.2 + 0.4j, 0.5 - 0.3j, 0.1 + 0.2j, 1.0 - 0.7j])
    base = np.empty(p.shape)
    base[0] = rho0
    for a in range(3):
        base[a + 1] = rho0 * U[a]
    base[4] = p0 / (gamma - 1) + 0.5 * rho0 * sum(v * v for v in U)
    delta = np.real(vhat[:, None, None, None] * np.exp(1j * k * X)[None])
    hcs = 1e-20
    dt, nsteps = 0.01, 12
    qn = O.run_c(p, dt, nsteps, base + 1j * hcs * delta)
    lin = np.imag(qn) / hcs
    h = 2 * np.pi / n[d]
    A = linearised_symbol(k, h, d, rho0, U, p0, gamma, mach, re, pr, viscous)
    Z = dt * A
    G = np.eye(5) + Z + Z @ Z / 2 + Z @ Z @ Z / 6
    amp = np.linalg.matrix_power(G, nsteps) @ vhat
    expect = np.real(amp[:, None, None, None] * np.exp(1j * k * X)[None])
    np.testing.assert_allclose(lin, expect, atol=1e-12 * np.abs(vhat).max())


# --------------------------------------------------------------------------
# Adjoint (reverse mode of the residual, the integrals and the time loop)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("visc", [1, 0])
def test_residual_adjoint_dot_product(visc):
    """<lam, J delta> = <J^T lam, delta>, with J delta taken by complex step
    of the residual (exact to rounding) -- an identity independent of how the
    transpose was written."""
    p = P((10, 12, 8), viscous=visc)
    q = S.random_state(p.n, 51, smooth=True)
    delta = S.random_field(p.shape, 52)
    lam = S.random_field(p.shape, 53)
    h = 1e-30
    Jd = np.imag(O.residual_c(p, q + 1j * h * delta)) / h
    JTl = O.residual_adjoint(p, q, lam)
    lhs = np.sum(lam * Jd)
    rhs = np.sum(JTl * delta)
    assert abs(lhs - rhs) <= 1e-12 * max(np.sum(np.abs(lam * Jd)), 1.0), (lhs, rhs)


def test_integrals_adjoint_matches_complex_step():
    p = P((10, 12, 8))
    q = S.random_state(p.n, 61, smooth=True)
    delta = S.random_field(p.shape, 62)
    h = 1e-30
    de = np.imag(O.integrals_c(p, q + 1j * h * delta)[2]) / h
    g = O.integrals_adjoint(p, q, 1.0)
    assert abs(np.sum(g * delta) - de) <= 1e-12 * abs(de)


def test_trajectory_gradient_matches_complex_step():
    """dJ/dQ0 of J = dt sum_n w_n eps^S(Q^n) (trapezoid) by store-all reverse
    mode, against the complex-step directional derivative of the forward run."""
    p = P(12)
    q0 = O.init(p)
    delta = S.random_field(p.shape, 71)
    dt, nsteps = 0.01, 6
    J, g = O.dissipation_grad(p, dt, nsteps, q0)
    h = 1e-30
    Jc = O.dissipation_c(p, dt, nsteps, q0 + 1j * h * delta)
    assert abs(Jc.real - J) <= 1e-14 * abs(J)
    dd = Jc.imag / h
    assert abs(np.sum(g * delta) - dd) <= 1e-11 * abs(dd), (np.sum(g * delta), dd)


@pytest.mark.parametrize("split", [1, 2, 3, 4, 5, 6])
def test_adjoint_refuses_other_split_forms(split):
    """The C routines of the reverse mode are the transpose of the Blaisdell
    residual only; they refuse any other split form themselves (status -1) and
    leave their outputs untouched."""
    p = P(8, split=split)
    q = S.random_state(p.n, 81, smooth=True)
    lam = S.random_field(p.shape, 82)
    qbar = np.full(p.shape, 7.0)
    with pytest.raises(ValueError):
        O.residual_adjoint(p, q, lam, qbar)
    assert np.all(qbar == 7.0)
    with pytest.raises(ValueError):
        O.dissipation_grad(p, 0.01, 1, O.init(p))
