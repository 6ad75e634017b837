"""Dense-matrix brute force of the residual -- TEST INFRASTRUCTURE ONLY.

A second, independent and deliberately naive evaluation of the same residual
as ``tgv_oracle.cpp`` for tiny grids (16^3): each 4th-order central operator
(Sec. 2.3.1) is an explicit dense n x n periodic circulant matrix built from
its stencil weights, and is applied along one axis with ``numpy.tensordot``.
No code is shared with the C++ oracle or with the GPU path.
"""
from __future__ import annotations

import numpy as np


def circulant(n: int, weights: dict, scale: float) -> np.ndarray:
    """Dense periodic matrix M with (M f)_i = scale * sum_s weights[s] f_{(i+s) mod n}."""
    M = np.zeros((n, n))
    for i in range(n):
        for s, w in weights.items():
            M[i, (i + s) % n] += w * scale
    return M


def d1_matrix(n: int, h: float) -> np.ndarray:
    return circulant(n, {-2: 1.0, -1: -8.0, 1: 8.0, 2: -1.0}, 1.0 / (12.0 * h))


def d2_matrix(n: int, h: float) -> np.ndarray:
    return circulant(n, {-2: -1.0, -1: 16.0, 0: -30.0, 1: 16.0, 2: -1.0}, 1.0 / (12.0 * h * h))


class Ops:
    """Axis operators on fields shaped (nz, ny, nx); axis 0 = x, 1 = y, 2 = z."""

    def __init__(self, n, L):
        self.D1 = [d1_matrix(n[d], L[d] / n[d]) for d in range(3)]
        self.D2 = [d2_matrix(n[d], L[d] / n[d]) for d in range(3)]

    @staticmethod
    def _apply(M, f, axis):
        ax = 2 - axis  # array axis of physical axis
        return np.moveaxis(np.tensordot(M, f, axes=([1], [ax])), 0, ax)

    def d1(self, f, axis):
        return self._apply(self.D1[axis], f, axis)

    def d2(self, f, axis):
        return self._apply(self.D2[axis], f, axis)


SPLIT = ("blaisdell", "divergence", "feiereisen", "jameson", "kgp", "kok", "keep")


def _pair(ops, A, B, d):
    """Quadratic split of D(A B): 1/2 [D(A B) + A D(B) + B D(A)]."""
    return 0.5 * (ops.d1(A * B, d) + A * ops.d1(B, d) + B * ops.d1(A, d))


def convective(ops, rho, u, phi, d, split):
    """Split form of D_d(rho u_d phi) by its pairing of the three factors;
    the cubic Kennedy-Gruber-Pirozzoli form through its identity with the
    pairings, KGP = (Blaisdell + Feiereisen + Jameson) / 2 - divergence / 2."""
    if split == "divergence":
        return ops.d1(rho * u[d] * phi, d)
    if split == "blaisdell":
        return _pair(ops, rho * phi, u[d], d)
    if split == "feiereisen":
        return _pair(ops, rho * u[d], phi, d)
    if split == "jameson":
        return _pair(ops, rho, u[d] * phi, d)
    return 0.5 * (_pair(ops, rho * phi, u[d], d) + _pair(ops, rho * u[d], phi, d)
                  + _pair(ops, rho, u[d] * phi, d)) - 0.5 * ops.d1(rho * u[d] * phi, d)


# ---------------------------------------------------------------------------
# Two-point flux form.  A 4th-order central first difference D f_i =
# (1/h) sum_l a_l (f_{i+l} - f_{i-l}), a_1 = 2/3, a_2 = -1/12, is also the
# difference of interface fluxes (F_{i+1/2} - F_{i-1/2}) / h with
#   F_{i+1/2} = 2 sum_l a_l sum_{m=0}^{l-1} F(X_{i-m}, X_{i-m+l}),
# where F(X_a, X_b) is a symmetric flux between two grid points.  Each split
# form of the convective term is defined by its two-point flux (Kok 2009;
# Kuya, Totani and Kawai 2018), an arithmetic mean of a factor over the two
# points written {f} = (f_a + f_b)/2:
#   divergence {rho u phi};  Blaisdell {rho phi}{u};  Feiereisen {rho u}{phi};
#   Jameson {rho}{u phi};    Kennedy-Gruber-Pirozzoli {rho}{u}{phi};
#   Kok: mass {rho u}, momentum {rho u}{u_a}, energy {rho u}({e} + K^)
#   KEEP: mass {rho}{u}, momentum {rho}{u}{u_a}, energy {rho}{u}({e} + K^)
# with e = p / ((gamma - 1) rho) and K^ = sum_a u_a(a) u_a(b) / 2, and the
# pressure fluxes {p} (momentum) and {p u} (energy), except that Kok and KEEP
# take the energy's pressure flux as (p_a u_b + p_b u_a)/2.  This evaluates
# the fluxes directly and shares nothing with the product-rule expansions the
# oracle codes.
# ---------------------------------------------------------------------------
A_COEF = ((1, 2.0 / 3.0), (2, -1.0 / 12.0))


def _at(f, axis, s):
    """f taken s points further along physical axis `axis` (periodic)."""
    return np.roll(f, -s, axis=2 - axis)


def flux_difference(flux, X, d, h):
    """(F_{i+1/2} - F_{i-1/2}) / h along axis d for the two-point flux
    `flux(Xa, Xb)` of the fields in dict X (arrays shaped (nz, ny, nx))."""
    def shifted(s):
        return {k: [_at(c, d, s) for c in v] if isinstance(v, list) else _at(v, d, s) for k, v in X.items()}

    F_half = 0.0
    for l, a in A_COEF:
        for m in range(l):
            F_half = F_half + 2.0 * a * flux(shifted(-m), shifted(l - m))
    return (F_half - _at(F_half, d, -1)) / h


def _two_point_fluxes(split, d):
    """The five two-point fluxes (rho, m1, m2, m3, rho E) along axis d,
    convective plus pressure, as functions of the point states Xa, Xb."""
    avg = lambda A, B, f: 0.5 * (f(A) + f(B))
    ud = lambda X: X["u"][d]

    def conv(A, B, phi):
        if split == "divergence":
            return avg(A, B, lambda X: X["rho"] * ud(X) * phi(X))
        if split == "blaisdell":
            return avg(A, B, lambda X: X["rho"] * phi(X)) * avg(A, B, ud)
        if split in ("feiereisen", "kok"):
            return avg(A, B, lambda X: X["rho"] * ud(X)) * avg(A, B, phi)
        if split == "jameson":
            return avg(A, B, lambda X: X["rho"]) * avg(A, B, lambda X: ud(X) * phi(X))
        return avg(A, B, lambda X: X["rho"]) * avg(A, B, ud) * avg(A, B, phi)   # kgp, keep

    def energy(A, B):
        if split not in ("kok", "keep"):
            return conv(A, B, lambda X: X["E"] / X["rho"]) + avg(A, B, lambda X: X["p"] * ud(X))
        khat = 0.5 * sum(A["u"][a] * B["u"][a] for a in range(3))
        mass = (avg(A, B, lambda X: X["rho"] * ud(X)) if split == "kok"
                else avg(A, B, lambda X: X["rho"]) * avg(A, B, ud))
        return (conv(A, B, lambda X: X["e"]) + mass * khat
                + 0.5 * (A["p"] * ud(B) + B["p"] * ud(A)))

    fl = [lambda A, B: conv(A, B, lambda X: 1.0)]
    for a in range(3):
        fl.append(lambda A, B, a=a: conv(A, B, lambda X: X["u"][a]) + (avg(A, B, lambda X: X["p"]) if a == d else 0.0))
    fl.append(energy)
    return fl


def residual(q, n, L, gamma, mach, re, pr, viscous=True, split="blaisdell", flux_form=None):
    """R = -C - P + V for Q = (rho, m1, m2, m3, rho E) shaped (5, nz, ny, nx).
    The convective and pressure terms come from the dense pairing products
    (the five pairing forms) or, with flux_form=True (always for Kok and
    KEEP), from the two-point fluxes above."""
    ops = Ops(n, L)
    rho, m, E = q[0], [q[1], q[2], q[3]], q[4]
    u = [m[a] / rho for a in range(3)]
    p = (gamma - 1.0) * (E - 0.5 * (m[0] * u[0] + m[1] * u[1] + m[2] * u[2]))
    T = gamma * mach ** 2 * p / rho
    R = np.zeros_like(q)
    if flux_form or split in ("kok", "keep"):
        X = {"rho": rho, "u": u, "p": p, "E": E, "e": p / ((gamma - 1.0) * rho)}
        for d in range(3):
            for f, flux in enumerate(_two_point_fluxes(split, d)):
                R[f] -= flux_difference(flux, X, d, L[d] / n[d])
    else:
        phis = [np.ones_like(rho), u[0], u[1], u[2], E / rho]
        for f, phi in enumerate(phis):
            R[f] -= sum(convective(ops, rho, u, phi, d, split) for d in range(3))
        for a in range(3):
            R[a + 1] -= ops.d1(p, a)
        R[4] -= sum(ops.d1(p * u[d], d) for d in range(3))
    if viscous:
        G = [[ops.d1(u[a], d) for d in range(3)] for a in range(3)]
        div = G[0][0] + G[1][1] + G[2][2]
        Vm = []
        for a in range(3):
            lap = sum(ops.d2(u[a], d) for d in range(3))
            X = ops.d2(u[a], a) + sum(ops.d1(ops.d1(u[d], d), a) for d in range(3) if d != a)
            Vm.append((lap + X / 3.0) / re)
            R[a + 1] += Vm[a]
        VE = sum(u[a] * Vm[a] for a in range(3))
        for a in range(3):
            for d in range(3):
                tau = (G[a][d] + G[d][a] - (2.0 / 3.0 if a == d else 0.0) * div) / re
                VE = VE + tau * G[a][d]
        kappa = 1.0 / ((gamma - 1.0) * mach ** 2 * pr * re)
        VE = VE + kappa * sum(ops.d2(T, d) for d in range(3))
        R[4] += VE
    return R


def dissipation(q, n, L, re):
    """eps^S = (1/Re) <|curl u|^2> with dense D1 matrices."""
    ops = Ops(n, L)
    u = [q[a + 1] / q[0] for a in range(3)]
    G = [[ops.d1(u[a], d) for d in range(3)] for a in range(3)]
    w1 = G[2][1] - G[1][2]
    w2 = G[0][2] - G[2][0]
    w3 = G[1][0] - G[0][1]
    return float(np.mean(w1 ** 2 + w2 ** 2 + w3 ** 2) / re)
