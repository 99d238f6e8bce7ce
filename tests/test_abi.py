"""The C-ABI library loads and exports every symbol the header declares; host-side
argument validation works without a GPU (no compute call is made here)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2210_04184_amd import nlpr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nlpr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nlpr_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 10
    lib = nlpr.load()
    out = subprocess.run(["nm", "-D", "--defined-only", nlpr.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (nlpr_\w+)", out))
    for n in names:
        assert n in exported, f"{n} declared in nlpr.h but not exported"
        assert hasattr(lib, n)
    assert sorted(nlpr.EXPORTED) == names


def test_status_strings():
    lib = nlpr.load()
    for code in range(7):
        s = lib.nlpr_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.nlpr_status_string(99).decode() == "unknown status"


def test_params_struct_layout_matches_header():
    # 12 x 32-bit fields, then 4 doubles at offset 48
    assert ctypes.sizeof(nlpr.Params) == 80
    assert nlpr.Params.lam.offset == 48
    assert nlpr.Params.h.offset == 72


def _create(**over):
    kw = dict(p=64, q=64, L=8, Lh=1, d=4, blur_radius=1, K=1, Sw=2, iters=3, flags=0,
              lam=1e-3, lam1=1.0, rho=1e-2, h=0.1)
    kw.update(over)
    r = kw["blur_radius"]
    prm = nlpr.Params(kw["p"], kw["q"], kw["L"], kw["Lh"], kw["d"], r, kw["K"], kw["Sw"],
                      kw["iters"], kw["flags"], kw.get("Ls", 0), kw.get("monitor_every", 0), kw["lam"],
                      kw["lam1"], kw["rho"], kw["h"])
    blur = np.ones((2 * r + 1, 2 * r + 1), np.float32)
    R = np.ones((kw["L"], kw["Lh"]), np.float32)
    h = ctypes.c_void_p()
    lib = nlpr.load()
    rc = lib.nlpr_plan_create(ctypes.byref(prm), blur.ctypes.data_as(ctypes.c_void_p),
                              R.ctypes.data_as(ctypes.c_void_p), None, ctypes.byref(h))
    return rc, h, lib.nlpr_last_error().decode()


@pytest.mark.parametrize("over,code", [
    (dict(p=100), nlpr.ERR_UNSUPPORTED_SHAPE),          # 100 = 2^2 5^2 is not 2^a 3^b
    (dict(q=18), nlpr.ERR_UNSUPPORTED_SHAPE),           # not a multiple of 4
    (dict(p=4), nlpr.ERR_UNSUPPORTED_SHAPE),            # below the minimum side
    (dict(d=3), nlpr.ERR_UNSUPPORTED_SHAPE),            # d does not divide 64
    (dict(K=5), nlpr.ERR_UNSUPPORTED_SHAPE),
    (dict(Sw=9), nlpr.ERR_UNSUPPORTED_SHAPE),
    (dict(Lh=17), nlpr.ERR_UNSUPPORTED_SHAPE),
    (dict(blur_radius=17), nlpr.ERR_UNSUPPORTED_SHAPE),
    (dict(flags=nlpr.LOCAL_WINDOW, Sw=2), nlpr.ERR_UNSUPPORTED_SHAPE),
    (dict(rho=0.0), nlpr.ERR_INVALID_ARG),
    (dict(lam=-1.0), nlpr.ERR_INVALID_ARG),
    (dict(lam1=0.0), nlpr.ERR_INVALID_ARG),
    (dict(h=0.0), nlpr.ERR_INVALID_ARG),
    (dict(iters=-1), nlpr.ERR_INVALID_ARG),
    (dict(d=0), nlpr.ERR_INVALID_ARG),
    (dict(rho=float("nan")), nlpr.ERR_INVALID_ARG),
    (dict(p=64, q=4096, K=4, Sw=8, d=1), nlpr.ERR_UNSUPPORTED_SHAPE),   # sweep tile exceeds LDS
    (dict(Ls=9), nlpr.ERR_UNSUPPORTED_SHAPE),                         # more basis rows than bands
    (dict(Ls=2), nlpr.ERR_INVALID_ARG),                               # Ls without a basis
    (dict(monitor_every=-1), nlpr.ERR_INVALID_ARG),
    (dict(flags=nlpr.FUSED_S, p=4096, q=64, d=4), nlpr.ERR_UNSUPPORTED_SHAPE),   # 8 (d+1) p > 64 KiB
    (dict(flags=nlpr.FUSED_S, p=1024, q=64, d=8), nlpr.ERR_UNSUPPORTED_SHAPE),   # 73728 B: just over
])
def test_invalid_parameters_are_rejected_on_the_host(over, code):
    rc, h, msg = _create(**over)
    assert rc == code, msg
    assert h.value is None
    assert msg


def test_null_arguments_are_rejected():
    lib = nlpr.load()
    h = ctypes.c_void_p()
    assert lib.nlpr_plan_create(None, None, None, None, ctypes.byref(h)) == nlpr.ERR_INVALID_ARG
    n = ctypes.c_size_t()
    assert lib.nlpr_workspace_size(None, ctypes.byref(n)) == nlpr.ERR_INVALID_ARG
    assert lib.nlpr_solve(None, None, None, None, None, 0, None) == nlpr.ERR_INVALID_ARG
    assert lib.nlpr_plan_destroy(None) == nlpr.OK


def test_basis_without_Ls_is_rejected():
    lib = nlpr.load()
    prm = nlpr.Params(64, 64, 8, 1, 4, 1, 1, 2, 3, 0, 0, 0, 1e-3, 1.0, 1e-2, 0.1)
    blur = np.ones((3, 3), np.float32)
    R = np.ones((8, 1), np.float32)
    E = np.ones((4, 8), np.float32)
    h = ctypes.c_void_p()
    rc = lib.nlpr_plan_create(ctypes.byref(prm), blur.ctypes.data_as(ctypes.c_void_p),
                              R.ctypes.data_as(ctypes.c_void_p), E.ctypes.data_as(ctypes.c_void_p),
                              ctypes.byref(h))
    assert rc == nlpr.ERR_INVALID_ARG


def test_batch_rejects_scenes_with_different_iteration_counts():
    lib = nlpr.load()
    prm = (nlpr.Params * 2)(nlpr.Params(64, 64, 8, 1, 4, 1, 1, 2, 3, 0, 0, 0, 1e-3, 1.0, 1e-2, 0.1),
                            nlpr.Params(64, 64, 8, 1, 4, 1, 1, 2, 4, 0, 0, 0, 1e-3, 1.0, 1e-2, 0.1))
    blur = np.ones((3, 3), np.float32)
    R = np.ones((8, 1), np.float32)
    ptrs = (ctypes.c_void_p * 2)(blur.ctypes.data, blur.ctypes.data)
    rs = (ctypes.c_void_p * 2)(R.ctypes.data, R.ctypes.data)
    h = ctypes.c_void_p()
    assert lib.nlpr_batch_create(2, prm, ptrs, rs, None, ctypes.byref(h)) == nlpr.ERR_INVALID_ARG
    assert lib.nlpr_batch_create(0, prm, ptrs, rs, None, ctypes.byref(h)) == nlpr.ERR_INVALID_ARG
    assert lib.nlpr_batch_destroy(None) == nlpr.OK
    # scenes must also share the monitor interval
    prm2 = (nlpr.Params * 2)(nlpr.Params(64, 64, 8, 1, 4, 1, 1, 2, 3, 0, 0, 1, 1e-3, 1.0, 1e-2, 0.1),
                             nlpr.Params(64, 64, 8, 1, 4, 1, 1, 2, 3, 0, 0, 2, 1e-3, 1.0, 1e-2, 0.1))
    assert lib.nlpr_batch_create(2, prm2, ptrs, rs, None, ctypes.byref(h)) == nlpr.ERR_INVALID_ARG
    assert "monitor_every" in lib.nlpr_last_error().decode()


def test_monitor_entry_points_reject_null_handles():
    lib = nlpr.load()
    n = ctypes.c_int32(-1)
    assert lib.nlpr_monitor(None, None, 0, ctypes.byref(n)) == nlpr.ERR_INVALID_ARG
    assert lib.nlpr_batch_monitor(None, 0, None, 0, ctypes.byref(n)) == nlpr.ERR_INVALID_ARG
    assert n.value == -1
