"""Precision study: every precision form's trajectory against an FP64 reference.

Runs the Taylor-Green vortex in each precision form on the GPU (through the
C-ABI) and measures, against the FP64 oracle trajectory computed on the host:
  * relative L2 error of each conserved field after the run,
  * relative L2 error of the change Q(t) - Q(0) (the mean of rho E ~ 178.6
    hides errors in Q itself),
  * maximum relative error of the K and eps^S histories,
  * the paper's accuracy metric (Sec. 4.2, error heat maps): the mean absolute
    difference of eps^S from the double-precision run over the samples.
It also times each form (Mpt.stage/s) so speedups can be read beside errors.

Usage (GPU): python studies/precision.py --n 64 --steps 200 --every 10
The oracle reference is feasible up to ~64^3 x a few hundred steps on the
host; with --reference dp the GPU FP64 path (validated against the oracle at
smaller sizes and on sampled points at full size) is the reference instead.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

FORMS = ["DP", "SPDP_C64", "SPDP_WK", "SPDP", "SP_DPC", "SP", "HPSP", "HPSP_BF16", "HPSP_WK", "HPSP_RESWK", "HP",
         "HP_C16"]


def run_form(form, n, dt, nsteps, every, mach=0.1, reynolds=1600.0):
    import torch
    from paper_2505_20911_amd import tgv
    from paper_2505_20911_amd.solver import TGVSolver
    p = tgv.Params(n=(n, n, n), mach=mach, reynolds=reynolds)
    s = TGVSolver(p, tgv.PRESETS[form])
    s.init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = s.run(nsteps, dt, every)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    q = s.q.to(torch.float64).cpu().numpy()
    return q, hist.cpu().numpy(), p.N * 3 * nsteps / (wall * 1e6)


def oracle_reference(n, dt, nsteps, every, mach=0.1):
    import oracle as O
    p = O.Params(n=(n, n, n), mach=mach)
    q0 = O.init(p)
    q, hist = O.run(p, dt, nsteps, q0, every=every)
    return q0, q, hist


def errors(q, hist, q0, qref, href):
    out = {}
    out["rel_l2_Q"] = [float(np.linalg.norm(q[f] - qref[f]) / np.linalg.norm(qref[f])) for f in range(5)]
    dq = []
    for f in range(5):
        dref = qref[f] - q0[f]
        nrm = np.linalg.norm(dref)
        dq.append(float(np.linalg.norm((q[f] - q0[f]) - dref) / nrm) if nrm > 0 else None)
    out["rel_l2_dQ"] = dq
    out["max_rel_K"] = float(np.max(np.abs(hist[:, 0] - href[:, 0]) / np.abs(href[:, 0])))
    out["max_rel_eps"] = float(np.max(np.abs(hist[:, 2] - href[:, 2]) / np.abs(href[:, 2])))
    out["mean_abs_deps"] = float(np.mean(np.abs(hist[:, 2] - href[:, 2])))
    out["finite"] = bool(np.all(np.isfinite(q)))
    return out


def study(n, nsteps, every, forms=FORMS, reference="oracle", dt=None, mach=0.1):
    dt = dt if dt is not None else 3.7e-3 * 32 / n
    if reference == "oracle":
        q0, qref, href = oracle_reference(n, dt, nsteps, every, mach)
    else:
        import oracle as O
        q0 = O.init(O.Params(n=(n, n, n), mach=mach))
        qref, href, _ = run_form("DP", n, dt, nsteps, every, mach)
    res = {}
    for form in forms:
        q, hist, rate = run_form(form, n, dt, nsteps, every, mach)
        res[form] = errors(q, hist, q0, qref, href)
        res[form]["mpt_stage_per_s"] = rate
        print(f"[study] {form} done: max rel eps {res[form]['max_rel_eps']:.2e}, {rate:.0f} Mpt.stage/s",
              file=sys.stderr, flush=True)
    return {"n": n, "steps": nsteps, "every": every, "dt": dt, "mach": mach, "reference": reference, "forms": res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--reference", choices=["oracle", "dp"], default="oracle")
    ap.add_argument("--forms", default=",".join(FORMS))
    ap.add_argument("--dt", type=float, default=None, help="default: 3.7e-3 * 32 / n (constant CFL)")
    ap.add_argument("--mach", type=float, default=0.1)
    a = ap.parse_args()
    out = study(a.n, a.steps, a.every, a.forms.split(","), a.reference, a.dt, a.mach)
    for f, r in out["forms"].items():
        print(f"{f:10s} relL2(dQ) rho {r['rel_l2_dQ'][0]:.2e} E {r['rel_l2_dQ'][4]:.2e}  "
              f"K {r['max_rel_K']:.2e}  eps {r['max_rel_eps']:.2e}  mean|deps| {r['mean_abs_deps']:.2e}  "
              f"{r['mpt_stage_per_s']:.0f} Mpt.stage/s", file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
