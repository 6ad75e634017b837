"""Writes the FP64 oracle's Taylor-Green trajectory summary used by the GPU
parity test at 256^3: the flow integrals every `every` steps and the state at
512 seeded sample points after the last step.  Calls only the oracle.

Usage: python tests/golden/make_tgv_history.py --n 256 --steps 200 --every 10
(about 75 s per step on 8 host cores at 256^3).  The run advances in chunks of
--chunk steps (a multiple of --every) and rewrites the file after each chunk,
so an interrupted run still leaves a complete, shorter trajectory; chunking
does not change the result (the step is deterministic and the history rows at
chunk seams coincide)."""
import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402

SAMPLE_SEED = 2505


def sample_indices(N):
    return np.sort(np.random.default_rng(SAMPLE_SEED).choice(N, 512, replace=False)).astype(np.int64)


def write(out, n, dt, steps, every, wall, hist, idx, qs):
    with open(out + ".tmp", "w") as fh:
        fh.write(f"# FP64 oracle, Taylor-Green vortex {n}^3 (Sec. 4.1 initial state, Re 1600, M 0.1, Pr 0.71,\n")
        fh.write(f"# gamma 1.4, (2 pi)^3), 4th-order scheme, RK3 (Sec. 3.1), dt {dt!r}, {steps} steps.\n")
        fh.write(f"# written by: python tests/golden/make_tgv_history.py --n {n} --steps {steps} --every {every}"
                 f"  ({wall:.0f} s)\n")
        fh.write(f"n {n}\ndt {dt!r}\nsteps {steps}\nevery {every}\n")
        fh.write("# history: step K K_rho epsS sum_rho sum_m1 sum_m2 sum_m3 sum_rhoE\n")
        for m, row in enumerate(hist):
            fh.write("H %d " % (m * every) + " ".join("%.17e" % v for v in row) + "\n")
        fh.write("# final state at sampled points: flat index rho m1 m2 m3 rhoE\n")
        for i, row in zip(idx, qs):
            fh.write("Q %d " % i + " ".join("%.17e" % v for v in row) + "\n")
    os.replace(out + ".tmp", out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--chunk", type=int, default=20)
    ap.add_argument("--out", default=None, help="output file (default: tgv<n>_dp_trajectory.txt beside this script)")
    a = ap.parse_args()
    n = a.n
    assert a.chunk % a.every == 0, "--chunk must be a multiple of --every"
    dt = 3.7e-3 * 32 / n  # constant CFL
    out = a.out or os.path.join(HERE, f"tgv{n}_dp_trajectory.txt")
    p = O.Params(n=(n, n, n))
    idx = sample_indices(p.N)
    t = time.time()
    q, hist, done = None, None, 0
    while done < a.steps:
        k = min(a.chunk, a.steps - done)
        q, h = O.run(p, dt, k, q, every=a.every)
        hist = h if hist is None else np.concatenate([hist, h[1:]])
        done += k
        write(out, n, dt, done, a.every, time.time() - t, hist, idx, q.reshape(5, -1)[:, idx].T)
        print("steps", done, "of", a.steps, "after", round(time.time() - t), "s", flush=True)
    wall = time.time() - t
    print("wrote", out, "in", wall, "s")


if __name__ == "__main__":
    main()
