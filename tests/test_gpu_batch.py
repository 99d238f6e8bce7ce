"""Batched multi-scene solve and graph replay.

A batch runs every stage as one launch over all scenes; each scene's arithmetic is the
single-scene arithmetic, so every scene of a batch must equal its own single-scene solve bit
for bit, and match the FP64 oracle like any solve.  Graph replays must equal eager solves.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import nlpr_oracle as o
from paper_2210_04184_amd import nlpr

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def mixed_scenes(iters=6):
    """Uneven sizes, band counts, guides, decimations, patch and window radii, including a
    scene without a search window and one whose rows need two float4 items per thread."""
    shapes = [  # p, q, L, Lh, d, r, K, Sw
        (64, 64, 8, 1, 4, 3, 1, 2),
        (48, 96, 5, 4, 4, 2, 2, 3),
        (36, 36, 3, 2, 2, 1, 1, 1),
        (32, 48, 4, 1, 4, 1, 1, 0),
        (16, 2048, 2, 1, 2, 1, 0, 2),
        (72, 72, 31, 4, 8, 4, 1, 1),
    ]
    return [synth.make_scene(synth.small_spec(p=p, q=q, L=L, Lh=Lh, d=d, blur_radius=r, K=K,
                                              Sw=Sw, iters=iters, seed=20 + i, tile=8))
            for i, (p, q, L, Lh, d, r, K, Sw) in enumerate(shapes)]


@pytest.mark.parametrize("flags", [0, nlpr.GRAPH])
def test_batch_equals_single_scene_solves(flags):
    scenes = mixed_scenes()
    batch = nlpr.Batch.from_scenes(scenes, flags=flags)
    Yls, Yhs = [dev(s.Yl) for s in scenes], [dev(s.Yh) for s in scenes]
    Zs, ws = batch.solve(Yls, Yhs)
    for i, sc in enumerate(scenes):
        plan = nlpr.Plan.from_scene(sc)
        Z, _ = plan.solve(Yls[i], Yhs[i])
        np.testing.assert_array_equal(host(Zs[i]), host(Z), err_msg=f"scene {i}")
    # a second call on the same workspace (graph replay when enabled) gives the same result
    Zs2, _ = batch.solve(Yls, Yhs, ws=ws)
    for a, b in zip(Zs, Zs2):
        assert torch.equal(a, b)


def test_batch_matches_oracle():
    scenes = mixed_scenes(iters=8)
    batch = nlpr.Batch.from_scenes(scenes, flags=nlpr.GRAPH)
    Zs, _ = batch.solve([dev(s.Yl) for s in scenes], [dev(s.Yh) for s in scenes])
    for i, sc in enumerate(scenes):
        ref = o.solve(sc.Yl.astype(np.float64), sc.Yh.astype(np.float64),
                      o.Problem.from_scene(sc), sc.spec.iters).X
        assert rel(host(Zs[i]), ref) <= 1e-4, i


def test_graph_replays_match_eager_with_work_in_between():
    sc = synth.make_scene(synth.config("c1", iters=12))
    eager = nlpr.Plan.from_scene(sc)
    Ze, _ = eager.solve(dev(sc.Yl), dev(sc.Yh))
    ref = host(Ze)
    g = nlpr.Plan.from_scene(sc, flags=nlpr.GRAPH)
    ws = g.alloc_workspace()
    Yl, Yh = dev(sc.Yl), dev(sc.Yh)
    for rep in range(4):
        Z, _ = g.solve(Yl, Yh, ws=ws)
        np.testing.assert_array_equal(host(Z), ref, err_msg=f"replay {rep}")
        junk = torch.randn(1 << 20, device="cuda")
        ws[: junk.numel()].copy_(junk.view(torch.uint8)[: junk.numel()])   # scribble on the state
        torch.cuda.synchronize()
    # other buffers (another scene of the same shape) through the same graph
    sc2 = synth.make_scene(synth.config("c1", iters=12, seed=9))
    Z2, _ = g.solve(dev(sc2.Yl), dev(sc2.Yh), ws=ws)
    Z2e, _ = eager.solve(dev(sc2.Yl), dev(sc2.Yh))
    np.testing.assert_array_equal(host(Z2), host(Z2e))


def test_c4_batch_sample_matches_oracle():
    """Scenes drawn like the 48-scene workload (128^2 and 192^2 here, so the oracle stays
    quick), 5 iterations."""
    specs = [s.replace(iters=5) for s in synth.batch_specs(48) if s.p <= 192][:4]
    scenes = [synth.make_scene(s) for s in specs]
    batch = nlpr.Batch.from_scenes(scenes, flags=nlpr.GRAPH)
    Zs, _ = batch.solve([dev(s.Yl) for s in scenes], [dev(s.Yh) for s in scenes])
    for i, sc in enumerate(scenes):
        ref = o.solve(sc.Yl.astype(np.float64), sc.Yh.astype(np.float64),
                      o.Problem.from_scene(sc), sc.spec.iters).X
        assert rel(host(Zs[i]), ref) <= 1e-4, (i, sc.spec)


@pytest.mark.parametrize("Lh", [1, 4, 16])
def test_threads_per_pixel_do_not_change_the_result(Lh):
    """A P-update launch over few pixels gives each pixel 4 threads (band shares added
    through LDS), one over many pixels 1 thread (the same shares added in registers).  Three
    256 x 192 scenes solved one at a time take the first form, together the second; both
    must give the same bits, with every guide-band class."""
    scenes = [synth.make_scene(synth.small_spec(p=256, q=192, L=7 + 3 * i, Lh=Lh, d=4,
                                                blur_radius=2, K=1, Sw=1, iters=3,
                                                seed=60 + i, tile=16))
              for i in range(3)]
    batch = nlpr.Batch.from_scenes(scenes)
    Yls, Yhs = [dev(s.Yl) for s in scenes], [dev(s.Yh) for s in scenes]
    Zs, _ = batch.solve(Yls, Yhs)
    for i, sc in enumerate(scenes):
        Z, _ = nlpr.Plan.from_scene(sc).solve(Yls[i], Yhs[i])
        np.testing.assert_array_equal(host(Zs[i]), host(Z), err_msg=f"scene {i}")
