"""Build libtgv.so (the HIP kernels and the C-ABI) in-tree for gfx950.

Each .hip source is compiled to an object with hipcc (in parallel), then the
objects are linked into paper_2505_20911_amd/libtgv.so.  The streaming
probes that the benchmark compares the step kernels with (stream_probe.hip)
go into a library of their own, libtgv_probe.so.  Packed-FP32 VALU
instructions are disabled for all device code, and multiply-add contraction is
limited to single source expressions (-ffp-contract=on) so that the same
expression rounds identically wherever it is inlined.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build", "libtgv")
LIB = os.path.join(PKG, "libtgv.so")
PROBE_LIB = os.path.join(PKG, "libtgv_probe.so")
ARCH = os.environ.get("TGV_OFFLOAD_ARCH", "gfx950")

SOURCES = ["abi.hip", "init.hip", "residual_tiled.hip", "rk_stage.hip", "integrals.hip", "adjoint.hip"]
PROBE_SOURCES = ["stream_probe.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are contracted only within one source expression, so a
    # computation rounds the same way in every kernel and unrolled copy
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    f"-I{INCLUDE}", f"-I{CSRC}",
]


# Per-source compiler options (none at present: the default scheduler keeps
# the adjoint gather within 2 waves' registers per SIMD in FP64, where the
# memory-clause scheduler spilled it).
EXTRA: dict[str, list[str]] = {}


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *CFLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    warn = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if verbose and warn:
        print(warn, flush=True)
    return obj


def _link(lib: str, objs: list[str], verbose: bool) -> None:
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = SOURCES + PROBE_SOURCES
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    _link(LIB, objs[:len(SOURCES)], verbose)
    _link(PROBE_LIB, objs[len(SOURCES):], verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
