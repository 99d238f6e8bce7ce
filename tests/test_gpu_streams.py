"""Calls on one plan from two streams, with separate workspaces, give the results each call
gives alone: the device work of successive calls on a plan runs in call order, so a call
never rewrites the plan's device descriptor while the previous call's kernels still read it."""
import numpy as np
import pytest
import torch

import synth
from paper_2210_04184_amd import nlpr

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_solves_and_forward_passes_on_two_streams():
    spec = synth.small_spec(p=128, q=192, L=16, Lh=2, d=4, blur_radius=3, K=1, Sw=2, iters=30,
                            seed=41)
    a, b = synth.make_scene(spec), synth.make_scene(spec, seed=42)
    print("[streams] 128x192x16, 30 iterations, two scenes on two streams", flush=True)
    plan = nlpr.Plan.from_scene(a)
    try:
        Yla, Yha, Ylb, Yhb = dev(a.Yl), dev(a.Yh), dev(b.Yl), dev(b.Yh)
        wsa, wsb = plan.alloc_workspace(), plan.alloc_workspace()
        Za_ref, _ = plan.solve(Yla, Yha, ws=wsa)
        Zb_ref, _ = plan.solve(Ylb, Yhb, ws=wsb)
        torch.cuda.synchronize()
        s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
        s1.wait_stream(torch.cuda.current_stream())
        s2.wait_stream(torch.cuda.current_stream())
        Za = torch.empty_like(Za_ref)
        Zb = torch.empty_like(Zb_ref)
        Zf = torch.empty_like(Zb_ref)
        ckb, _ = plan.grad_sizes()
        ck = torch.empty(ckb, dtype=torch.uint8, device="cuda")
        for _ in range(3):
            plan.solve(Yla, Yha, Z=Za, ws=wsa, stream=s1)
            plan.solve(Ylb, Yhb, Z=Zb, ws=wsb, stream=s2)
            plan.solve(Yla, Yha, Z=Za, ws=wsa, stream=s1)
            plan.forward(Ylb, Yhb, Z=Zf, ws=wsb, ck=ck, stream=s2)
        torch.cuda.synchronize()
        assert torch.equal(Za, Za_ref)
        assert torch.equal(Zb, Zb_ref)
        assert torch.equal(Zf, Zb_ref)
    finally:
        plan.close()


def test_side_stream_overlap_is_bit_identical():
    """A scene of 2^22 pixel-bands runs blur, P-update and B^T W1 + W2 of each iteration on a
    second stream while the sweep runs; a plan with stage timers keeps one stream.  Both
    give the same bits (the assembly adds the same terms in the same order), also through a
    captured graph, on the caller's own stream."""
    spec = synth.small_spec(p=128, q=128, L=256, Lh=2, d=4, blur_radius=3, K=1, Sw=2, iters=4,
                            seed=43)
    sc = synth.make_scene(spec)
    print("[streams] 128x128x256 (2^22 pixel-bands), side stream against one stream", flush=True)
    Yl, Yh = dev(sc.Yl), dev(sc.Yh)
    out = {}
    for name, flags in (("one stream", nlpr.TIMING), ("side stream", 0),
                        ("graph", nlpr.GRAPH)):
        plan = nlpr.Plan.from_scene(sc, flags=flags)
        try:
            s = torch.cuda.Stream()
            s.wait_stream(torch.cuda.current_stream())
            Z, ws = plan.solve(Yl, Yh, stream=s)
            torch.cuda.synchronize()
            out[name] = (Z.clone(), plan.region_view(ws, nlpr.REGION_C).clone(),
                         plan.region_view(ws, nlpr.REGION_LAMBDA2).clone())
            del Z, ws
        finally:
            plan.close()
    ref = out["one stream"]
    assert bool(torch.isfinite(ref[0]).all())
    for name in ("side stream", "graph"):
        for a, b in zip(out[name], ref):
            assert torch.equal(a, b), name
