"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no arithmetic of the method: it only draws seeded random
arrays (NumPy PCG64 via ``numpy.random.default_rng``) in the shapes and value
ranges of the Taylor-Green workload, so that the oracle and the GPU path see
identical bytes.  Layout: conserved vector Q shaped (5, nz, ny, nx), x fastest;
velocity-like fields shaped (3, nz, ny, nx).
"""
from __future__ import annotations

import numpy as np


def state_shape(n):
    nx, ny, nz = n
    return (5, nz, ny, nx)


def random_state(n, seed: int, smooth: bool = False) -> np.ndarray:
    """A generic conserved state with positive density and pressure.

    rho in [0.9, 1.1], momenta in [-0.25, 0.25], rho E in [177.5, 178.5]
    (the magnitudes of the M = 0.1 Taylor-Green state, where rho E is about 178.6).
    ``smooth=True`` draws a few low Fourier modes per field instead of
    white noise (still non-symmetric, so no symmetry of the grid is hit).
    """
    rng = np.random.default_rng(seed)
    nx, ny, nz = n
    shape = (nz, ny, nx)
    if not smooth:
        u01 = rng.random((5,) + shape)
    else:
        z, y, x = np.meshgrid(np.arange(nz) * 2 * np.pi / nz, np.arange(ny) * 2 * np.pi / ny,
                              np.arange(nx) * 2 * np.pi / nx, indexing="ij")
        u01 = np.empty((5,) + shape)
        for f in range(5):
            acc = np.zeros(shape)
            for _ in range(4):
                kx, ky, kz = rng.integers(0, 3, size=3)
                ph = rng.random(3) * 2 * np.pi
                acc += np.cos(kx * x + ph[0]) * np.cos(ky * y + ph[1]) * np.cos(kz * z + ph[2])
            u01[f] = 0.5 + acc / 8.0  # in [0, 1]
    q = np.empty((5,) + shape)
    q[0] = 0.9 + 0.2 * u01[0]
    q[1:4] = 0.5 * (u01[1:4] - 0.5)
    q[4] = 177.5 + u01[4]
    return np.ascontiguousarray(q)


def random_field(shape, seed: int) -> np.ndarray:
    """Standard normal array of the given shape (adjoint seeds, directions)."""
    return np.random.default_rng(seed).standard_normal(shape)


def directions(n, seed: int) -> np.ndarray:
    """Gaussian velocity direction d_s shaped (3, nz, ny, nx), unnormalised, FP64."""
    nx, ny, nz = n
    return np.random.default_rng(seed).standard_normal((3, nz, ny, nx))
