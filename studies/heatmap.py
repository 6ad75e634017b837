"""Time-step and Mach-number sweeps of the precision forms (paper Sec. 4.2,
the two error heat maps): each form's dissipation history against the
double-precision run with the same parameters, measured by the paper's metric,
the mean absolute difference of eps^S sampled every 0.5 time units of
simulated time (t = 0, 0.5, ..., 20), and by the maximum relative difference.

  dt sweep:   M = 0.5, Re = 800, dt in {0.01, 0.005, 0.0025, 0.00125, 0.000625}, t = 20 (20/dt steps)
  Mach sweep: dt = 0.000625, Re = 800, M in {0.1, 0.2, 0.3, 0.4, 0.5}, 32000 steps (t = 20)

on the periodic (2 pi)^3 Taylor-Green vortex at n^3 (default 128^3, the
resolution of the paper's 64^3 symmetric box; its 256^3 symmetric box, 512^3
here, is out of reach for 10 x 12 runs of up to 32000 steps: the precision
behaviour, not the resolution, is what is compared).

Usage (GPU): python studies/heatmap.py [--n 128] [--forms SP,HPSP,...] > heatmap.json
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from studies.precision import FORMS, run_form  # noqa: E402

DTS = [0.01, 0.005, 0.0025, 0.00125, 0.000625]
MACHS = [0.1, 0.2, 0.3, 0.4, 0.5]


SAMPLE_T = 0.5  # the paper's sampling interval of eps^S, in time units


def sweep(n, cases, forms):
    out = []
    for mach, dt, nsteps in cases:
        every = int(round(SAMPLE_T / dt))
        _, href, _ = run_form("DP", n, dt, nsteps, every, mach, 800.0)
        row = {"mach": mach, "dt": dt, "steps": nsteps, "every": every, "samples": int(href.shape[0]),
               "dp_eps_mean": float(np.mean(href[:, 2])), "forms": {}}
        for form in forms:
            if form == "DP":
                continue
            _, h, rate = run_form(form, n, dt, nsteps, every, mach, 800.0)
            d = np.abs(h[:, 2] - href[:, 2])
            row["forms"][form] = {"mean_abs_deps": float(np.mean(d)),
                                  "max_rel_deps": float(np.max(d / np.abs(href[:, 2]))),
                                  "finite": bool(np.all(np.isfinite(h))), "mpt_stage_per_s": rate}
        out.append(row)
        print(f"[heatmap] M={mach} dt={dt} steps={nsteps}: " + "  ".join(
            f"{f} {r['mean_abs_deps']:.1e}" for f, r in row["forms"].items()), file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--forms", default=",".join(FORMS))
    ap.add_argument("--sweeps", default="dt,mach")
    a = ap.parse_args()
    forms = a.forms.split(",")
    sweeps = a.sweeps.split(",")
    dt_cases = [(0.5, dt, int(round(20.0 / dt))) for dt in DTS]
    mach_cases = [(m, 0.000625, 32000) for m in MACHS]
    res = {"n": a.n, "reynolds": 800.0, "sample_every_time_units": SAMPLE_T}
    if "dt" in sweeps:
        res["dt_sweep"] = sweep(a.n, dt_cases, forms)
    if "mach" in sweeps:
        res["mach_sweep"] = sweep(a.n, mach_cases, forms)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
