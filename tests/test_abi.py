"""C-ABI contract checks that need no GPU: the library loads, exports every
function include/tgv.h declares, and rejects bad arguments on the host
(validation runs before any HIP call) with the documented codes and a message."""
import ctypes
import os
import re

import pytest

from paper_2505_20911_amd import tgv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tgv.h")

NS_ERR_ARG, NS_ERR_DTYPE, NS_ERR_SHAPE, NS_ERR_ALIGN = -1, -2, -3, -4


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|size_t|char\s*\*|void)\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = tgv.load()
    names = declared_functions()
    assert len(names) >= 12, names
    for name in names:
        assert hasattr(lib, name), f"libtgv.so does not export {name}"
    assert set(names) == set(tgv._EXPORTS), "binding and header disagree"


def test_abi_version():
    assert tgv.tgv_abi_version() == 2


def _call_residual(params, prec, q=0x1000, r=0x2000):
    lib = tgv.load()
    return lib.ns_residual(ctypes.byref(params.c()), ctypes.byref(prec.c()), ctypes.c_void_p(q),
                           ctypes.c_void_p(r), None)


@pytest.mark.parametrize("n", [(4, 8, 8), (8, 4, 8), (8, 8, 2), (0, 8, 8)])
def test_rejects_grids_below_stencil_width(n):
    assert _call_residual(tgv.Params(n=n), tgv.PRESETS["DP"]) == NS_ERR_SHAPE
    assert "< 5" in tgv.ns_last_error()


def test_rejects_unsupported_precision_forms():
    bad = [tgv.Prec(tgv.f16, tgv.f64, tgv.f64, tgv.f64), tgv.Prec(tgv.f64, tgv.f64, tgv.f64, tgv.f16),
           tgv.Prec(tgv.f32, tgv.f32, tgv.f32, tgv.bf16), tgv.Prec(tgv.bf16, tgv.bf16, tgv.bf16, tgv.f32),
           tgv.Prec(tgv.f64, tgv.f64, tgv.f16, tgv.f16), tgv.Prec(tgv.f64, tgv.f32, tgv.f32, tgv.f32)]
    for prec in bad:
        assert _call_residual(tgv.Params(n=(8, 8, 8)), prec) == NS_ERR_DTYPE
        assert "unsupported precision form" in tgv.ns_last_error()


def test_rejects_null_and_misaligned_and_aliased_pointers():
    p, prec = tgv.Params(n=(8, 8, 8)), tgv.PRESETS["DP"]
    lib = tgv.load()
    assert lib.ns_residual(ctypes.byref(p.c()), ctypes.byref(prec.c()), None, ctypes.c_void_p(0x2000),
                           None) == NS_ERR_ARG
    assert "q is NULL" in tgv.ns_last_error()
    assert _call_residual(p, prec, q=0x1008) == NS_ERR_ALIGN
    assert _call_residual(p, prec, q=0x1000, r=0x1000) == NS_ERR_ARG
    assert lib.ns_residual(None, ctypes.byref(prec.c()), ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000),
                           None) == NS_ERR_ARG


def test_rejects_bad_scalars():
    lib = tgv.load()
    prec = tgv.PRESETS["DP"]
    for kw in ({"gamma": 1.0}, {"mach": 0.0}, {"reynolds": -1.0}, {"prandtl": float("nan")},
               {"viscous": 2}, {"L": (6.28, 0.0, 6.28)}):
        p = tgv.Params(n=(8, 8, 8), **kw)
        assert _call_residual(p, prec) == NS_ERR_ARG, kw
    p = tgv.Params(n=(8, 8, 8))
    for stage in (-1, 3):
        assert lib.rk_stage(ctypes.byref(p.c()), ctypes.byref(prec.c()), stage, 0.1, ctypes.c_void_p(0x1000),
                            ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000), None) == NS_ERR_ARG
    assert lib.rk_stage(ctypes.byref(p.c()), ctypes.byref(prec.c()), 0, float("inf"), ctypes.c_void_p(0x1000),
                        ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000), None) == NS_ERR_ARG


def test_adjoint_forms_and_workspace_sizes():
    p = tgv.Params(n=(8, 10, 12))
    assert tgv.ns_residual_adjoint_workspace_bytes(p, tgv.PRESETS["DP"]) == 15 * p.N * 8
    assert tgv.ns_residual_adjoint_workspace_bytes(p, tgv.PRESETS["SP"]) == 15 * p.N * 4
    assert tgv.ns_residual_adjoint_workspace_bytes(p, tgv.PRESETS["HPSP"]) == 0  # unsupported form
    assert tgv.flow_integrals_adjoint_workspace_bytes(p, tgv.PRESETS["DP"]) == 3 * p.N * 8
    assert tgv.flow_integrals_workspace_bytes(p) >= 8 * 8
    lib = tgv.load()
    rc = lib.ns_residual_adjoint(ctypes.byref(p.c()), ctypes.byref(tgv.PRESETS["HPSP"].c()),
                                 ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000),
                                 ctypes.c_void_p(0x4000), None)
    assert rc == NS_ERR_DTYPE


def test_python_binding_refuses_host_tensors():
    import torch
    p = tgv.Params(n=(8, 8, 8))
    q = torch.zeros(p.shape, dtype=torch.float64)
    with pytest.raises(ValueError, match="GPU tensor"):
        tgv.ns_residual(p, tgv.PRESETS["DP"], q, q.clone())


def test_split_form_validation():
    """Split forms other than Blaisdell exist for the DP and HPSP forms only;
    the adjoint rejects them; out-of-range values are rejected -- all before
    any HIP call (host validation, runs without a GPU)."""
    lib = tgv.load()
    dummy = [ctypes.c_void_p(0x1000 * (i + 1)) for i in range(4)]
    p_sp = tgv.Params(n=(8, 8, 8), split=tgv.SPLIT_FORMS["kgp"])
    for form in ("SP", "SPDP", "HP"):
        rc = lib.ns_residual(ctypes.byref(p_sp.c()), ctypes.byref(tgv.PRESETS[form].c()), dummy[0], dummy[1], None)
        assert rc == NS_ERR_ARG, form
        rc = lib.ns_residual_rk_stage(ctypes.byref(p_sp.c()), ctypes.byref(tgv.PRESETS[form].c()), 0, 1e-3,
                                      dummy[0], dummy[1], dummy[2], None)
        assert rc == NS_ERR_ARG, form
    rc = lib.ns_residual_adjoint(ctypes.byref(p_sp.c()), ctypes.byref(tgv.PRESETS["DP"].c()), dummy[0], dummy[1],
                                 dummy[2], dummy[3], None)
    assert rc == NS_ERR_ARG and b"Blaisdell" in lib.ns_last_error()
    bad = tgv.Params(n=(8, 8, 8), split=7)
    rc = lib.ns_residual(ctypes.byref(bad.c()), ctypes.byref(tgv.PRESETS["DP"].c()), dummy[0], dummy[1], None)
    assert rc == NS_ERR_ARG and b"split" in lib.ns_last_error()


def test_last_error_is_per_thread():
    """ns_last_error() is thread-local: a failing call on one thread does not
    overwrite the message another thread is about to read."""
    import threading
    lib = tgv.load()
    msgs = {}
    gate = threading.Barrier(2)

    def worker(name, n):
        p = tgv.Params(n=(n, 8, 8))
        gate.wait()
        rc = lib.ns_residual(ctypes.byref(p.c()), ctypes.byref(tgv.PRESETS["DP"].c()), ctypes.c_void_p(0x1001),
                             ctypes.c_void_p(0x2000), None)
        gate.wait()
        msgs[name] = (rc, lib.ns_last_error())

    ts = [threading.Thread(target=worker, args=("shape", 3)), threading.Thread(target=worker, args=("align", 8))]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert msgs["shape"][0] == NS_ERR_SHAPE and b"n[0]" in msgs["shape"][1]
    assert msgs["align"][0] == NS_ERR_ALIGN and b"aligned" in msgs["align"][1]


def test_stream_probe_library_loads_and_validates_on_the_host():
    """The benchmark's streaming probes live in libtgv_probe.so, apart from the
    method's library; bad arguments are rejected before any launch."""
    path = os.path.join(ROOT, "paper_2505_20911_amd", "libtgv_probe.so")
    lib = ctypes.CDLL(path)
    lib.tgv_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_ulonglong, ctypes.c_void_p]
    lib.tgv_probe_stage_stream.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int] + [ctypes.c_void_p] * 4
    assert lib.tgv_probe_copy(None, ctypes.c_void_p(0x1000), 16, None) == -1
    assert lib.tgv_probe_copy(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 24, None) == -1  # not 16-byte
    assert lib.tgv_probe_copy(ctypes.c_void_p(0x1008), ctypes.c_void_p(0x2000), 32, None) == -1  # misaligned
    assert lib.tgv_probe_copy(ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), 0, None) == 0  # nothing to do
    a, b, c = (ctypes.c_void_p(0x1000 * k) for k in (1, 2, 3))
    assert lib.tgv_probe_stage_stream(0, 16, 8, a, b, c, None) == -1
    assert lib.tgv_probe_stage_stream(64, 0, 8, a, b, c, None) == -1
    assert lib.tgv_probe_stage_stream(64, 16, 3, a, b, c, None) == -1
    assert lib.tgv_probe_stage_stream(64, 16, 8, None, b, c, None) == -1


def test_grid_size_limits_are_validated_before_launch():
    """N <= 2^34 is accepted by the parameter check (the element-wise kernels
    loop grid-stride, so no 1-D dispatch limit applies); larger grids are
    refused with NS_ERR_SHAPE before any HIP call (the pointers here are never
    touched).  The tiled launches (at most 2^34 / (256 x 128) blocks of 256 or
    512 threads for the plane marches) stay below the 2^32 work-items of one
    dispatch for every grid that passes this check."""
    lib = tgv.load()
    prec = tgv.PRESETS["DP"]
    big = tgv.Params(n=(4096, 4096, 1025))  # 2^34 + 2^24 points
    assert _call_residual(big, prec) == NS_ERR_SHAPE
    assert "2^34" in tgv.ns_last_error()
    for fn, args in (("ns_residual_adjoint", [ctypes.c_void_p(0x1000 * (i + 1)) for i in range(4)]),
                     ("flow_integrals_adjoint", [ctypes.c_void_p(0x1000), ctypes.c_double(1.0),
                                                 ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)])):
        rc = getattr(lib, fn)(ctypes.byref(big.c()), ctypes.byref(prec.c()), *args, None)
        assert rc == NS_ERR_SHAPE, fn
        assert "2^34" in tgv.ns_last_error()


def test_noalloc_integrals_refuse_grids_beyond_the_static_scratch():
    lib = tgv.load()
    prec = tgv.PRESETS["DP"]
    # 1088 x 1024 x 1024: 17 x 256 x 16 = 69632 first-pass blocks > 65536 rows
    p = tgv.Params(n=(1088, 1024, 1024))
    rc = lib.flow_integrals_noalloc(ctypes.byref(p.c()), ctypes.byref(prec.c()), ctypes.c_void_p(0x1000),
                                    ctypes.c_void_p(0x2000), None)
    assert rc == NS_ERR_SHAPE
    assert "static scratch" in tgv.ns_last_error()
    assert tgv.flow_integrals_workspace_bytes(p) > 4 << 20
    # 1024^3 fits exactly (65536 rows, 4 MiB)
    assert tgv.flow_integrals_workspace_bytes(tgv.Params(n=(1024, 1024, 1024))) == 4 << 20
    rc = lib.flow_integrals_noalloc(ctypes.byref(p.c()), ctypes.byref(prec.c()), None, ctypes.c_void_p(0x2000), None)
    assert rc == NS_ERR_ARG


def test_state_map_and_trapezoid_validate_on_the_host():
    lib = tgv.load()
    p = tgv.Params(n=(8, 8, 8))
    a, b, c, d = (ctypes.c_void_p(x) for x in (0x1000, 0x2000, 0x3000, 0x4000))
    assert lib.ns_state_from_velocity(ctypes.byref(p.c()), tgv.NS_F16, a, b, c, d, None) == NS_ERR_DTYPE
    assert lib.ns_state_from_velocity(ctypes.byref(p.c()), tgv.NS_F64, a, b, c, a, None) == NS_ERR_ARG
    assert lib.ns_state_from_velocity(ctypes.byref(p.c()), tgv.NS_F64, None, b, c, d, None) == NS_ERR_ARG
    assert lib.ns_state_from_velocity_adjoint(ctypes.byref(p.c()), tgv.NS_F64, a, b, c,
                                              ctypes.c_void_p(0x4008), None) == NS_ERR_ALIGN
    assert lib.tgv_init_primitive(ctypes.byref(tgv.Params(n=(4, 8, 8)).c()), tgv.NS_F64, a, b, c, None) == NS_ERR_SHAPE
    assert lib.dissipation_trapezoid(a, 0, 8, 2, 1e-3, b, None) == NS_ERR_ARG
    assert lib.dissipation_trapezoid(a, 5, 8, 8, 1e-3, b, None) == NS_ERR_ARG
    assert lib.dissipation_trapezoid(None, 5, 8, 2, 1e-3, b, None) == NS_ERR_ARG
