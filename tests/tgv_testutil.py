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
