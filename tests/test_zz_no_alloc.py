"""nlpr_solve_noalloc, the solve whose workspace is the library's static device array,
against nlpr_solve with a caller workspace: two calls in a row, the second on a smaller
scene, each bit-for-bit equal to nlpr_solve and within 1e-4 relative RMSE of the FP64
oracle; plans too large for the array and plans with flags it does not take are refused."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from oracle import nlpr_oracle as o
from paper_2210_04184_amd import nlpr

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _noalloc(plan, Yl, Yh, Z):
    """Straight through the C ABI."""
    lib = nlpr.load()
    return lib.nlpr_solve_noalloc(plan.handle, ctypes.c_void_p(Yl.data_ptr()),
                                  ctypes.c_void_p(Yh.data_ptr()), ctypes.c_void_p(Z.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_noalloc_solve_equals_solve_on_two_calls_in_a_row():
    specs = [synth.small_spec(p=64, q=96, L=10, Lh=2, d=4, blur_radius=3, K=1, Sw=2, iters=12,
                              seed=61),
             synth.small_spec(p=48, q=64, L=5, Lh=1, d=2, blur_radius=2, K=1, Sw=1, iters=9,
                              seed=62)]
    for spec in specs:
        sc = synth.make_scene(spec)
        print(f"[noalloc] {spec.p}x{spec.q}x{spec.L}, {spec.iters} iterations", flush=True)
        plan = nlpr.Plan.from_scene(sc)
        try:
            assert plan.workspace_bytes <= nlpr.NOALLOC_WORKSPACE_BYTES
            Yl, Yh = dev(sc.Yl), dev(sc.Yh)
            Z = torch.full((spec.L, spec.p, spec.q), float("nan"), device="cuda")
            assert _noalloc(plan, Yl, Yh, Z) == nlpr.OK
            Zref, _ = plan.solve(Yl, Yh)
            torch.cuda.synchronize()
            assert torch.equal(Z, Zref)
            ref = o.solve(sc.Yl, sc.Yh, o.Problem.from_scene(sc), spec.iters).X
            z = Z.cpu().numpy().astype(np.float64)
            rel = float(np.linalg.norm(z - ref) / np.linalg.norm(ref))
            print(f"[noalloc] relRMSE vs FP64 oracle = {rel:.3e}", flush=True)
            assert rel <= 1e-4
        finally:
            plan.close()


def test_noalloc_refuses_what_it_cannot_run():
    big = synth.small_spec(p=256, q=256, L=31, Lh=3, d=4, K=1, Sw=1, iters=2, seed=63)
    sc = synth.make_scene(big)
    plan = nlpr.Plan.from_scene(sc)
    Yl, Yh = dev(sc.Yl), dev(sc.Yh)
    Z = torch.empty((big.L, big.p, big.q), device="cuda")
    try:
        assert plan.workspace_bytes > nlpr.NOALLOC_WORKSPACE_BYTES
        assert _noalloc(plan, Yl, Yh, Z) == nlpr.ERR_WORKSPACE_TOO_SMALL
        assert b"static workspace" in nlpr.load().nlpr_last_error()
    finally:
        plan.close()
    small = synth.small_spec(p=32, q=32, L=4, Lh=1, d=4, K=1, Sw=1, iters=2, seed=64)
    sc = synth.make_scene(small)
    for flag in (nlpr.STATE_IN, nlpr.GRAPH, nlpr.TIMING):
        plan = nlpr.Plan.from_scene(sc, flags=flag)
        try:
            Z = torch.empty((small.L, small.p, small.q), device="cuda")
            assert _noalloc(plan, dev(sc.Yl), dev(sc.Yh), Z) == nlpr.ERR_INVALID_ARG
        finally:
            plan.close()
