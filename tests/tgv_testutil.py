"""Shared helpers of the test-suite (tolerances, dtype plumbing)."""
import numpy as np
import torch

UNIT_ROUNDOFF = {torch.float64: 2.0 ** -53, torch.float32: 2.0 ** -24, torch.float16: 2.0 ** -11,
                 torch.bfloat16: 2.0 ** -8}


def oracle_params(p):
    """oracle.Params with the same grid and physics as a binding Params."""
    import oracle as O
    return O.Params(n=tuple(p.n), L=tuple(p.L), gamma=p.gamma, mach=p.mach, re=p.reynolds, pr=p.prandtl,
                    viscous=p.viscous, split=p.split)


def term_scale(n, L, gamma, q):
    """Per-field magnitude of the individual flux-derivative terms of the
    residual, (max|q_f| (1 + max|u|) + max|p|) / h_min.  Rounding errors of any
    evaluation order are relative to this scale, not to R itself (at the
    Taylor-Green state R_E is a cancellation of terms ~|rho E|/h down to O(1))."""
    rho, m, E = q[0], q[1:4], q[4]
    umax = np.abs(m / rho).max()
    pmax = np.abs((gamma - 1) * (E - 0.5 * (m * m).sum(0) / rho)).max()
    h = min(L[d] / n[d] for d in range(3))
    return np.array([(np.abs(q[f]).max() * (1 + umax) + pmax) / h for f in range(5)])


def rounded(q64: np.ndarray, dtype: torch.dtype) -> torch.Tensor:
    """The FP64 array rounded to a storage dtype on the host (an input, shared
    bit-for-bit by the oracle -- after exact widening -- and the GPU)."""
    return torch.from_numpy(np.ascontiguousarray(q64)).to(dtype)


def widened(t: torch.Tensor) -> np.ndarray:
    return t.detach().to("cpu").to(torch.float64).numpy()


def adjoint_term_scale(p, q, rbar):
    """Magnitude bound of the individual terms of the residual adjoint
    Q_bar = (dR/dQ)^T R_bar at state q (one scale for all five outputs, since
    the chain through u = m / rho and p = (gamma-1)(rho E - |m|^2 / (2 rho))
    mixes every field into every output).  With |D1 f| <= (3/2) max|f| / h and
    |D2 f| <= (16/3) max|f| / h^2 (the sums of the stencil weights' magnitudes)
    over three directions:
      convection and pressure: 3 (3/2) / h * A (sum_f max|q_f| + max|p|) (1 + U) / rho_min,
      viscous stress and work: 3 (16/3) / h^2 * A (1 + U)^2 / (Re rho_min),
      heat flux:               3 (16/3) / h^2 * A kappa (max T + gamma M^2) / rho_min,
    A = max|R_bar|, U = max|u|, h the smallest spacing.  Rounding errors of any
    evaluation order of the adjoint are relative to this scale."""
    rho, m, E = q[0], q[1:4], q[4]
    gamma, mach, re, pr = p.gamma, p.mach, p.reynolds, p.prandtl
    A = np.abs(rbar).max()
    U = np.abs(m / rho).max()
    pr_ = (gamma - 1) * (E - 0.5 * (m * m).sum(0) / rho)
    T = gamma * mach * mach * pr_ / rho
    h = min(p.L[d] / p.n[d] for d in range(3))
    rmin = rho.min()
    kappa = 1.0 / ((gamma - 1) * mach * mach * pr * re)
    conv = 4.5 / h * A * (sum(np.abs(q[f]).max() for f in range(5)) + np.abs(pr_).max()) * (1 + U) / rmin
    visc = 16.0 / h ** 2 * A * (1 + U) ** 2 / (re * rmin) if p.viscous else 0.0
    heat = 16.0 / h ** 2 * A * kappa * (np.abs(T).max() + gamma * mach * mach) / rmin if p.viscous else 0.0
    return conv + visc + heat
