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
