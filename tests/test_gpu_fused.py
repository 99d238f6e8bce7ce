"""GPU fused-S splitting: S B kept in the X-subproblem, solved per aliasing group of d^2
frequencies, against the oracle's fused mode (a dense d^2 x d^2 FP64 solve per group).

Tolerances.  One X-update is held to 2e-5 relative RMSE: two FP32 FFTs plus the
Sherman-Morrison correction, which near the zero frequency cancels up to a factor
(rho d^2 + sum |b^|^2 / a) / (rho d^2) of its terms.  Whole solves are held to the 1e-4
relative RMSE bar on Z.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import nlpr_oracle as o
from paper_2210_04184_amd import nlpr

pytestmark = pytest.mark.gpu

SHAPES = {
    # name: (p, q, L, Lh, d, blur_radius, K, Sw)
    "c1": (64, 64, 8, 1, 4, 3, 1, 2),
    "ragged": (72, 96, 5, 2, 4, 2, 2, 3),
    "radix3_d2": (48, 36, 3, 3, 2, 1, 1, 1),
    "radix3_d3": (48, 36, 3, 1, 3, 1, 1, 1),
    "d8": (64, 128, 4, 4, 8, 4, 1, 2),
    "d1": (32, 48, 3, 1, 1, 2, 1, 1),
}


def scene_for(name, iters=10, seed=21):
    p, q, L, Lh, d, r, K, Sw = SHAPES[name]
    if name == "c1":
        return synth.make_scene(synth.config("c1", iters=iters))
    return synth.make_scene(synth.small_spec(p=p, q=q, L=L, Lh=Lh, d=d, blur_radius=r, K=K,
                                             Sw=Sw, iters=iters, seed=seed, tile=8))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def fused_problem(sc, **kw):
    return o.Problem.from_scene(sc, fused=True, **kw)


@pytest.mark.parametrize("name", list(SHAPES))
def test_fused_xsolve_stage_matches_oracle(name):
    sc = scene_for(name)
    plan = nlpr.Plan.from_scene(sc, flags=nlpr.FUSED_S)
    pr = fused_problem(sc)
    rng = np.random.default_rng(3)
    C = rng.standard_normal((sc.spec.L, sc.spec.p, sc.spec.q)).astype(np.float32)
    X = torch.empty(C.shape, device="cuda")
    plan.stage(nlpr.STAGE_XSOLVE, [dev(C), X, plan.alloc_workspace()])
    a = o.fused_denominator(pr.p, pr.q, pr.window, pr.K)
    want = o.x_update_fused(C.astype(np.float64), pr, a)
    assert rel(host(X), want) <= 2e-5


@pytest.mark.parametrize("name", list(SHAPES))
def test_fused_solve_matches_oracle(name):
    sc = scene_for(name, iters=10)
    plan = nlpr.Plan.from_scene(sc, flags=nlpr.FUSED_S)
    Z, _ = plan.solve(dev(sc.Yl), dev(sc.Yh))
    ref = o.solve(sc.Yl.astype(np.float64), sc.Yh.astype(np.float64), fused_problem(sc),
                  sc.spec.iters)
    assert rel(host(Z), ref.X) <= 1e-4


def test_fused_solve_c1_fifty_iterations_with_monitor():
    sc = scene_for("c1", iters=50)
    plan = nlpr.Plan.from_scene(sc, flags=nlpr.FUSED_S, monitor_every=10)
    Z, _ = plan.solve(dev(sc.Yl), dev(sc.Yh))
    ref = o.solve(sc.Yl.astype(np.float64), sc.Yh.astype(np.float64), fused_problem(sc), 50,
                  monitor_every=10)
    assert rel(host(Z), ref.X) <= 1e-4
    got = plan.monitor()
    assert [int(g[0]) for g in got] == [10, 20, 30, 40, 50]
    xn = float(np.linalg.norm(ref.X))
    for g, w in zip(got, ref.monitor):
        for k, f in enumerate(("objective", "data_l", "data_h", "reg"), start=1):
            assert g[k] == pytest.approx(getattr(w, f), rel=1e-4), f
        assert g[5] == 0.0 and w.r1 == 0.0
        assert abs(g[6] - w.r2) <= 1e-4 * w.r2 + 1e-5 * xn


def test_fused_resume_and_batch_are_bit_exact():
    scs = [scene_for("ragged", iters=6), scene_for("d8", iters=6)]
    plan = nlpr.Plan.from_scene(scs[0], flags=nlpr.FUSED_S)
    Yl, Yh = dev(scs[0].Yl), dev(scs[0].Yh)
    Zfull, _ = plan.solve(Yl, Yh)
    p4 = nlpr.Plan.from_scene(scs[0], flags=nlpr.FUSED_S, iters=4)
    Z4, ws = p4.solve(Yl, Yh)
    p2 = nlpr.Plan.from_scene(scs[0], flags=nlpr.FUSED_S | nlpr.STATE_IN, iters=2)
    Zr, _ = p2.solve(Yl, Yh, Z=Z4, ws=ws)
    assert torch.equal(Zr, Zfull)
    batch = nlpr.Batch.from_scenes(scs, flags=nlpr.FUSED_S | nlpr.GRAPH)
    Zb, _ = batch.solve([dev(s.Yl) for s in scs], [dev(s.Yh) for s in scs])
    for s, zb in zip(scs, Zb):
        z, _ = nlpr.Plan.from_scene(s, flags=nlpr.FUSED_S).solve(dev(s.Yl), dev(s.Yh))
        assert torch.equal(z, zb)


def test_fused_and_paper_splitting_approach_each_other_at_the_oracle_rate():
    # both splittings minimise the same objective (Theorem 1 for each), so their iterates
    # approach each other; ADMM does so slowly (sublinearly), and the GPU distance after T
    # iterations must match the FP64 oracle's distance after T iterations
    sc = scene_for("radix3_d2", iters=300)
    Yl, Yh = dev(sc.Yl), dev(sc.Yh)
    za, _ = nlpr.Plan.from_scene(sc, rho=0.05).solve(Yl, Yh)
    zb, _ = nlpr.Plan.from_scene(sc, flags=nlpr.FUSED_S, rho=0.05).solve(Yl, Yh)
    got = rel(host(za), host(zb))
    Yl64, Yh64 = sc.Yl.astype(np.float64), sc.Yh.astype(np.float64)
    a = o.solve(Yl64, Yh64, o.Problem.from_scene(sc, rho=0.05), 300).X
    b = o.solve(Yl64, Yh64, o.Problem.from_scene(sc, rho=0.05, fused=True), 300).X
    want = rel(a, b)
    assert want < 1e-2                     # far closer than after a few iterations (6e-2 at 5)
    assert abs(got - want) <= 0.05 * want + 1e-5
