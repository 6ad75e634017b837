"""The committed rocprofv3 summaries the benchmark reads: the HBM counter
bytes of the residual kernels (profiles/hbm_traffic.json) must have been
taken on the current kernel source, else the benchmark's roofline reports
no traffic; and counter bytes cannot fall below the bytes the kernel must
move (5N(2|Tq| + |Tq~|) at stage 0, 5N(2|Tq| + 2|Tq~|) at stages 1-2)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_profile_matches_kernel_source():
    with open(bench.TRAFFIC_FILE) as fh:
        d = json.load(fh)
    assert d["kernel_source_sha256"] == bench.kernel_source_sha256(), \
        "kernel source changed since profiles/hbm_traffic.json was taken: re-run the counters"
    assert bench.measured_traffic("ns_residual_rk_stage/DP/512") is not None


def test_fused_dp_traffic_covers_algorithmic_bytes():
    n = 512 ** 3
    algorithmic = 5 * n * (2 * 8 + 8 + 2 * (2 * 8 + 2 * 8)) / 3  # mean over the three stages
    traffic = bench.measured_traffic("ns_residual_rk_stage/DP/512")
    assert algorithmic <= traffic <= 1.5 * algorithmic, (traffic, algorithmic)
