"""Throughput of the explicit RK3 time step on the Taylor-Green vortex.

One step = three RK stages, each one fused residual evaluation and one
two-register update, plus the FP64 flow integrals every 10 steps (paper
Sec. 3.1 and Sec. 4.1).  Reported as grid-point RK-stage updates per second
(Mpt.stage/s = N * 3 * steps / wall time) on one GPU, with the residual
kernel's achieved algorithmic bandwidth against the HBM peak, and the FP64
CPU oracle timed on a bounded sample beside it.

Usage: python bench.py [--steps K] [--warmup W] [--n 512] [--forms DP,SPDP,...]
Prints exactly one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Mpt·stage/s + % HBM peak, TGV 512^3: FP64 vs half-single/single-double"
HBM_PEAK_GBS = 8000.0
ALL_FORMS = ["DP", "SPDP", "SPDP_C64", "SP_DPC", "SP", "HPSP", "HPSP_BF16", "HP"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--forms", default=",".join(ALL_FORMS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=128, help="grid of the oracle sample")
    return ap.parse_args()


def nbytes(dtype):
    import torch
    return torch.empty((), dtype=dtype).element_size()


def time_form(form, n, steps, warmup, dt):
    import torch
    from paper_2505_20911_amd import tgv
    from paper_2505_20911_amd.solver import TGVSolver

    prec = tgv.PRESETS[form]
    p = tgv.Params(n=(n, n, n))
    s = TGVSolver(p, prec)
    s.init()
    every = 10
    hist = torch.empty((steps // every + 2, 8), dtype=torch.float64, device="cuda")
    for w in range(warmup):
        s.step(dt)
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    res_ev, rk_ev = [], []
    t_start, t_end = ev(), ev()
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    t_start.record(stream)
    row = 0
    for k in range(steps):
        if k % every == 0:
            s.integrals(hist[row])
            row += 1
        for i in range(3):
            a, b, c = ev(), ev(), ev()
            a.record(stream)
            tgv.ns_residual(p, prec, s.q, s.r)
            b.record(stream)
            tgv.rk_stage(p, prec, i, dt, s.q, s.qt, s.r)
            c.record(stream)
            res_ev.append((a, b))
            rk_ev.append((b, c, i))
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = t_start.elapsed_time(t_end)
    res_ms = [a.elapsed_time(b) for a, b in res_ev]
    rk_ms = [(b.elapsed_time(c), i) for b, c, i in rk_ev]
    finite = bool(torch.isfinite(hist[:row]).all())
    N = p.N
    bq, bqt, br = nbytes(prec.q), nbytes(prec.qt), nbytes(prec.r)
    res_bytes = 5 * N * (bq + br)
    rk_bytes = {0: 5 * N * (br + 2 * bq + bqt), 1: 5 * N * (br + 2 * bq + 2 * bqt), 2: 5 * N * (br + 2 * bq + 2 * bqt)}
    res_avg = sum(res_ms) / len(res_ms)
    rk_avg = sum(t for t, _ in rk_ms) / len(rk_ms)
    rk_gbs = sum(rk_bytes[i] / (t * 1e-3) for t, i in rk_ms) / len(rk_ms) / 1e9
    out = {
        "mpt_stage_per_s": N * 3 * steps / (wall * 1e6),
        "ms_per_step": 1e3 * wall / steps,
        "gpu_ms_per_step": gpu_ms / steps,
        "residual_ms": res_avg,
        "residual_bytes_per_launch": res_bytes,
        "residual_gbs": res_bytes / (res_avg * 1e-3) / 1e9,
        "rk_stage_ms": rk_avg,
        "rk_stage_gbs": rk_gbs,
        "finite": finite,
        "K_first": float(hist[0, 0]),
    }
    del s, hist
    torch.cuda.empty_cache()
    return out


def cpu_baseline(n):
    """One RK3 step (three residual + stage pairs) of the FP64 oracle on an
    n^3 Taylor-Green grid: same per-point work as the GPU workload, sized to
    a few tens of seconds on the host cores."""
    import numpy as np
    import oracle as O
    cores = len(os.sched_getaffinity(0))
    os.environ.setdefault("OMP_NUM_THREADS", str(cores))
    p = O.Params(n=(n, n, n))
    q = O.init(p)
    t0 = time.perf_counter()
    O.run(p, 2.3125e-4 * 512 / n, 1, q)
    wall = time.perf_counter() - t0
    return {"value": p.N * 3 / (wall * 1e6), "unit": "Mpt·stage/s",
            "cores": int(os.environ.get("OMP_NUM_THREADS", cores)), "kind": "oracle",
            "sample": f"one RK3 step (3 stages) of the FP64 oracle on a {n}^3 TGV grid, {wall:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU slab "
              "decomposition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2505_20911_amd import tgv
    tgv.load()
    n = args.n
    dt = 3.7e-3 * 32 / n
    forms = [f for f in args.forms.split(",") if f]
    results = {}
    for f in forms:
        print(f"[bench] {f} {n}^3: {args.warmup} warmup + {args.steps} timed steps", file=sys.stderr, flush=True)
        results[f] = time_form(f, n, args.steps, args.warmup, dt)
        print(f"[bench] {f}: {results[f]['mpt_stage_per_s']:.0f} Mpt.stage/s, residual "
              f"{results[f]['residual_ms']:.3f} ms ({results[f]['residual_gbs']:.0f} GB/s)",
              file=sys.stderr, flush=True)
    head = results.get("DP") or results[forms[0]]
    head_form = "DP" if "DP" in results else forms[0]
    for f, r in results.items():
        r["speedup_vs_DP"] = r["mpt_stage_per_s"] / results["DP"]["mpt_stage_per_s"] if "DP" in results else None
    line = {
        "metric": METRIC,
        "value": head["mpt_stage_per_s"],
        "unit": "Mpt·stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head_form == "DP" else head_form,
        "data": "synthetic",
        "config": {"workload": f"Taylor-Green vortex, periodic (2pi)^3, {n}^3 points, Re=1600, M=0.1, "
                               f"{head_form} form, RK3 dt={dt:.6g}, integrals every 10 steps",
                   "grid": [n, n, n], "form": head_form},
        "roofline": {"bound": "hbm", "kernel": "ns_residual",
                     "achieved": head["residual_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": head["residual_gbs"] / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": head["residual_bytes_per_launch"],
                     "avg_launch_ms": head["residual_ms"]},
        "forms": results,
    }
    if not args.no_cpu_baseline:
        print(f"[bench] cpu baseline: oracle on {args.cpu_n}^3", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args.cpu_n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
