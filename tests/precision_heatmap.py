"""Time-step and Mach-number sweeps of the precision forms (paper Sec. 4.2,
the two error heat maps): each form's dissipation history against the
double-precision run with the same parameters, measured by the paper's metric,
the mean absolute difference of eps^S over the samples, and by the maximum
relative difference.

  dt sweep:   M = 0.5, Re = 800, dt in {0.01, 0.005, 0.0025, 0.00125, 0.000625}, t = 20 (20/dt steps)
  Mach sweep: dt = 0.000625, Re = 800, M in {0.1, 0.2, 0.3, 0.4, 0.5}, 32000 steps (t = 20)

on the periodic (2 pi)^3 Taylor-Green vortex at n^3 (default 64^3: the
paper's 256^3 symmetric box is out of reach for 2 x 5 x 8 runs of up to 32000
steps; the precision behaviour, not the resolution, is what is compared).

Usage (GPU): python tests/precision_heatmap.py [--n 64] [--every 100] > heatmap.json
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import numpy as np  # noqa: E402

from precision_study import FORMS, run_form  # noqa: E402

DTS = [0.01, 0.005, 0.0025, 0.00125, 0.000625]
MACHS = [0.1, 0.2, 0.3, 0.4, 0.5]


def sweep(n, every, cases, forms):
    out = []
    for mach, dt, nsteps in cases:
        _, href, _ = run_form("DP", n, dt, nsteps, every, mach, 800.0)
        row = {"mach": mach, "dt": dt, "steps": nsteps, "forms": {}}
        for form in forms:
            if form == "DP":
                continue
            _, h, rate = run_form(form, n, dt, nsteps, every, mach, 800.0)
            d = np.abs(h[:, 2] - href[:, 2])
            row["forms"][form] = {"mean_abs_deps": float(np.mean(d)),
                                  "max_rel_deps": float(np.max(d / np.abs(href[:, 2]))),
                                  "finite": bool(np.all(np.isfinite(h)))}
        out.append(row)
        print(f"[heatmap] M={mach} dt={dt} steps={nsteps}: " + "  ".join(
            f"{f} {r['mean_abs_deps']:.1e}" for f, r in row["forms"].items()), file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--forms", default=",".join(FORMS))
    a = ap.parse_args()
    forms = a.forms.split(",")
    dt_cases = [(0.5, dt, int(round(20.0 / dt))) for dt in DTS]
    mach_cases = [(m, 0.000625, 32000) for m in MACHS]
    res = {"n": a.n, "reynolds": 800.0, "every": a.every,
           "dt_sweep": sweep(a.n, a.every, dt_cases, forms),
           "mach_sweep": sweep(a.n, a.every, mach_cases, forms)}
    print(json.dumps(res))


if __name__ == "__main__":
    main()
