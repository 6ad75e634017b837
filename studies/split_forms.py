"""Robustness of the split forms in the inviscid limit (paper Sec. 4.2, the
split-form comparison): inviscid Taylor-Green vortex, 64^3, M = 0.4,
dt = 0.004, to t = 20 (5000 steps), each split form in double precision and in
half-single, with the kinetic energy history K(t)/K(0).  Without viscosity the
discrete kinetic energy should stay at 1; forms that do not control aliasing
grow and diverge.  Reports, per form and precision, K/K0 at the end (or where
the run stopped) and the first time K/K0 leaves [0.5, 1.5] or turns
non-finite.

Usage (GPU): python studies/split_forms.py [--n 64] [--steps 5000] > split.json
"""
import argparse
import json
import math
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def run(split, form, n, steps, dt, every):
    import torch
    from paper_2505_20911_amd import tgv
    from paper_2505_20911_amd.solver import TGVSolver
    p = tgv.Params(n=(n, n, n), mach=0.4, viscous=0, split=split)
    s = TGVSolver(p, tgv.PRESETS[form])
    s.init()
    hist = s.run(steps, dt, every).cpu().numpy()
    K = hist[:, 1] / hist[0, 1]  # K_rho, the kinetic energy the inviscid equations conserve
    t = [m * every * dt for m in range(len(K))]
    blow = next((t[m] for m in range(len(K)) if not math.isfinite(K[m]) or not 0.5 < K[m] < 1.5), None)
    last = next((m for m in range(len(K) - 1, -1, -1) if math.isfinite(K[m])), 0)
    return {"t": t, "K_over_K0": [float(x) for x in K], "diverged_at": blow,
            "final": float(K[-1]) if math.isfinite(K[-1]) else None, "last_finite_t": t[last]}


def main():
    from paper_2505_20911_amd import tgv
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--dt", type=float, default=0.004)
    ap.add_argument("--every", type=int, default=50)
    a = ap.parse_args()
    out = {"n": a.n, "steps": a.steps, "dt": a.dt, "mach": 0.4, "viscous": 0, "runs": {}}
    for name, split in tgv.SPLIT_FORMS.items():
        for form in ("DP", "HPSP"):
            r = run(split, form, a.n, a.steps, a.dt, a.every)
            out["runs"][f"{name}/{form}"] = r
            print(f"[split] {name:10s} {form:5s} K/K0 final {r['final']}  left [0.5, 1.5] at t = {r['diverged_at']}",
                  file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
