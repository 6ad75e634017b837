"""The allocation-free flow integrals (flow_integrals_noalloc: the partial sums
in the library's static device scratch, no workspace argument) against the
workspace entry point flow_integrals, through the C-ABI, on two calls in a
row: a large grid, then a smaller one (the second must not see the first
call's rows).  Both run the same kernels in the same order, so the eight
integrals must agree bitwise; they are also checked against the FP64 oracle
within the integrals' parity bound (1e-12 relative, or absolute on the scale
of <|m|> for the momentum means, which cancel to ~0)."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle as O
import tgv_synth as S
from paper_2505_20911_amd import tgv
from tgv_testutil import oracle_params, rounded

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _both(p, prec, q64):
    q = rounded(q64, prec.q).cuda()
    out_ws = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    out_na = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    ws = torch.empty(tgv.flow_integrals_workspace_bytes(p) // 8, dtype=torch.float64, device="cuda")
    tgv.flow_integrals(p, prec, q, ws, out_ws)
    lib = tgv.load()
    rc = lib.flow_integrals_noalloc(ctypes.byref(p.c()), ctypes.byref(prec.c()), ctypes.c_void_p(q.data_ptr()),
                                    ctypes.c_void_p(out_na.data_ptr()),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, tgv.ns_last_error()
    torch.cuda.synchronize()
    return out_ws.cpu().numpy(), out_na.cpu().numpy(), q


def _check_oracle(p, q, got):
    ref = O.integrals(oracle_params(p), q.cpu().to(torch.float64).numpy())
    for m in (0, 1, 2, 3, 7):
        assert abs(got[m] - ref[m]) <= 1e-12 * abs(ref[m]), (m, got[m], ref[m])
    mscale = np.abs(q[1:4].cpu().to(torch.float64).numpy()).mean()
    assert np.all(np.abs(got[4:7] - ref[4:7]) <= 1e-13 * mscale), (got[4:7], ref[4:7])


@pytest.mark.parametrize("form", ["DP", "SP", "HP"])
def test_noalloc_integrals_equal_workspace_entry_point(form):
    prec = tgv.PRESETS[form]
    first, second = (130, 72, 96), (24, 20, 16)
    results = []
    for n, seed in ((first, 11), (second, 12)):
        say("noalloc integrals", form, n)
        p = tgv.Params(n=n)
        q64 = S.random_state(n, seed, smooth=True)
        ws, na, q = _both(p, prec, q64)
        assert np.all(np.isfinite(na)), na
        assert np.array_equal(ws, na), (ws, na)
        _check_oracle(p, q, na)
        results.append(na)
    assert not np.array_equal(results[0], results[1])


def test_noalloc_integrals_wrapper_and_full_size_launch():
    # the binding's wrapper, and the largest grid the scratch holds along one
    # axis pattern the benchmark uses (512^3 DP: 8192 first-pass rows)
    n = (512, 512, 512)
    say("noalloc integrals 512^3 DP")
    p = tgv.Params(n=n)
    prec = tgv.PRESETS["DP"]
    q = torch.empty(p.shape, dtype=torch.float64, device="cuda")
    tgv.tgv_init(p, q)
    out_ws = torch.empty(8, dtype=torch.float64, device="cuda")
    out_na = torch.empty(8, dtype=torch.float64, device="cuda")
    ws = torch.empty(tgv.flow_integrals_workspace_bytes(p) // 8, dtype=torch.float64, device="cuda")
    tgv.flow_integrals(p, prec, q, ws, out_ws)
    tgv.flow_integrals_noalloc(p, prec, q, out_na)
    torch.cuda.synchronize()
    a, b = out_ws.cpu().numpy(), out_na.cpu().numpy()
    assert np.array_equal(a, b), (a, b)
    assert abs(b[0] - 0.125) <= 1e-14 and abs(b[1] - 0.125) <= 1e-14
