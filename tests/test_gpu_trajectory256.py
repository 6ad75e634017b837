"""The 256^3 double-precision run against the FP64 oracle's stored trajectory
(`tests/golden/tgv256_dp_trajectory.txt`, written by the committed script
beside it, which calls only the oracle): flow integrals every 10 steps and the
final state at 512 seeded sample points.  Same physics, scheme and constant-CFL
dt as the benchmark, fused residual + RK stage path."""
import os
import sys

import numpy as np
import pytest
import torch

from paper_2505_20911_amd import tgv
from paper_2505_20911_amd.solver import TGVSolver

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tgv256_dp_trajectory.txt")


def load_golden():
    meta, hist, pts = {}, [], []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            tok = line.split()
            if tok[0] == "H":
                hist.append([float(v) for v in tok[2:]])
            elif tok[0] == "Q":
                pts.append([float(v) for v in tok[1:]])
            else:
                meta[tok[0]] = float(tok[1])
    pts = np.array(pts)
    return meta, np.array(hist), pts[:, 0].astype(np.int64), pts[:, 1:]


def test_trajectory_256_matches_oracle():
    meta, h_ref, idx, q_ref = load_golden()
    n, steps, every, dt = int(meta["n"]), int(meta["steps"]), int(meta["every"]), meta["dt"]
    print("trajectory", n, steps, dt, flush=True)
    sys.stdout.flush()
    p = tgv.Params(n=(n, n, n))
    s = TGVSolver(p, tgv.PRESETS["DP"])
    s.init()
    hist = s.run(steps, dt, every=every).cpu().numpy()
    got = s.q.reshape(5, -1)[:, torch.from_numpy(idx).to(s.q.device)].T.cpu().numpy()
    for m in (0, 1, 2):  # K, K_rho, eps^S
        rel = np.abs(hist[:, m] - h_ref[:, m]) / np.abs(h_ref[:, m])
        assert rel.max() <= 1e-12, (m, rel.max())
    # conserved totals: mass and energy to rounding of the sums, momentum stays ~0
    assert np.all(np.abs(hist[:, 3] - h_ref[:, 3]) <= 1e-13 * np.abs(h_ref[:, 3]))
    assert np.all(np.abs(hist[:, 7] - h_ref[:, 7]) <= 1e-13 * np.abs(h_ref[:, 7]))
    assert np.all(np.abs(hist[:, 4:7] - h_ref[:, 4:7]) <= 1e-13 * np.abs(h_ref[:, 3:4]))
    # scale of each field's rounding: its own magnitude, except that the three
    # momentum components share the magnitude of the momentum vector (w-momentum
    # starts at zero and stays far smaller than the others over the run, but is
    # computed from the O(1) components and rounds at their level)
    scale = np.abs(q_ref).max(0)
    scale[1:4] = scale[1:4].max()
    err = np.abs(got - q_ref).max(0)
    print("sampled final state error / field max", err / scale, flush=True)
    assert np.all(err <= 1e-12 * scale), err / scale
