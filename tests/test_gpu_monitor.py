"""GPU monitor: the objective of eq. (mainoptim) with its terms and the primal residuals of
eq. (fusionoptim), recorded every N iterations inside the solve, against the FP64 oracle's
records of the same iterations on the same float32 inputs.

Tolerances.  The GPU iterates differ from the oracle's by a relative RMSE of about 1e-7, and
each term is a sum of squares or absolute values of FP32 quantities accumulated in FP64, so
the objective terms are held to 1e-4 relative.  The residuals are differences of two
iterates of similar size; they are held to 1e-4 relative plus an absolute floor of 1e-5
times the norm of the iterate they are measured against.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import nlpr_oracle as o
from paper_2210_04184_amd import nlpr

pytestmark = pytest.mark.gpu

TERMS = ("objective", "data_l", "data_h", "reg")


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def scene(p, q, L, Lh, d, r, K, Sw, iters, seed=11, **kw):
    return synth.make_scene(synth.small_spec(p=p, q=q, L=L, Lh=Lh, d=d, blur_radius=r, K=K,
                                             Sw=Sw, iters=iters, seed=seed, tile=8, **kw))


def oracle_records(sc, every, E=None, **prkw):
    pr = o.Problem.from_scene(sc, E=None if E is None else E.astype(np.float64), **prkw)
    res = o.solve(sc.Yl.astype(np.float64), sc.Yh.astype(np.float64), pr, sc.spec.iters,
                  monitor_every=every)
    return res, pr


def check_records(got, res, pr):
    want = res.monitor
    assert got.shape == (len(want), nlpr.MON_RECORD)
    for g, w in zip(got, want):
        assert g[0] == w.iteration
        for k, name in enumerate(TERMS, start=1):
            assert g[k] == pytest.approx(getattr(w, name), rel=1e-4), name
        assert g[7] == 0.0
    # residual floors: the size of B X (for r1) and of X (for r2) at the last iterate
    xn = float(np.linalg.norm(res.X))
    bxn = float(np.linalg.norm(o.blur(res.X, pr.b)))
    for g, w in zip(got, want):
        assert abs(g[5] - w.r1) <= 1e-4 * w.r1 + 1e-5 * bxn
        assert abs(g[6] - w.r2) <= 1e-4 * w.r2 + 1e-5 * xn


@pytest.mark.parametrize("shape", [
    (64, 64, 8, 1, 4, 3, 1, 2),     # PAN guide, 3x3 patch, 5x5 window
    (72, 96, 5, 2, 4, 2, 2, 3),     # ragged sweep and monitor tiles
    (48, 36, 3, 3, 2, 1, 1, 1),     # radix-3 sizes, q < 64
])
def test_monitor_matches_oracle(shape):
    sc = scene(*shape, iters=10)
    plan = nlpr.Plan.from_scene(sc, monitor_every=3)
    plan.solve(dev(sc.Yl), dev(sc.Yh))
    got = plan.monitor()
    res, pr = oracle_records(sc, 3)
    assert [int(g[0]) for g in got] == [3, 6, 9, 10]
    check_records(got, res, pr)


@pytest.mark.parametrize("variant", ["unweighted", "local", "no_reg"])
def test_monitor_variants_match_oracle(variant):
    flags, prkw, shape = 0, {}, (64, 64, 4, 2, 4, 2, 1, 2)
    if variant == "unweighted":
        flags, prkw = nlpr.UNWEIGHTED, dict(unweighted=True)
    elif variant == "local":
        flags, prkw, shape = nlpr.LOCAL_WINDOW, dict(local=True), (64, 64, 4, 2, 4, 2, 1, 1)
    else:
        shape = (64, 64, 4, 2, 4, 2, 1, 0)          # Sw = 0: no regulariser term
    sc = scene(*shape, iters=6)
    plan = nlpr.Plan.from_scene(sc, flags=flags, monitor_every=2)
    plan.solve(dev(sc.Yl), dev(sc.Yh))
    got = plan.monitor()
    res, pr = oracle_records(sc, 2, **prkw)
    check_records(got, res, pr)
    if variant == "no_reg":
        assert np.all(got[:, 4] == 0.0)


def test_monitor_with_a_subspace_basis_matches_oracle():
    sc = scene(48, 96, 9, 4, 4, 2, 2, 3, iters=8, seed=31)
    E = np.random.default_rng(5).uniform(-1, 1, (3, 9)).astype(np.float32)
    plan = nlpr.Plan.from_scene(sc, E=E, monitor_every=4)
    plan.solve(dev(sc.Yl), dev(sc.Yh))
    res, pr = oracle_records(sc, 4, E=E)
    check_records(plan.monitor(), res, pr)


def test_monitor_leaves_the_solve_unchanged_and_repeats_bit_for_bit():
    sc = scene(72, 96, 5, 2, 4, 2, 2, 3, iters=7)
    Yl, Yh = dev(sc.Yl), dev(sc.Yh)
    Z0, _ = nlpr.Plan.from_scene(sc).solve(Yl, Yh)
    plan = nlpr.Plan.from_scene(sc, monitor_every=2)
    Z1, ws = plan.solve(Yl, Yh)
    first = plan.monitor()
    Z2, _ = plan.solve(Yl, Yh, ws=ws)
    assert torch.equal(Z0, Z1) and torch.equal(Z1, Z2)
    assert np.array_equal(first, plan.monitor())
    # the same records when the solve is replayed from a HIP graph
    gplan = nlpr.Plan.from_scene(sc, flags=nlpr.GRAPH, monitor_every=2)
    for _ in range(3):
        Z3, _ = gplan.solve(Yl, Yh)
        torch.cuda.synchronize()
        assert torch.equal(Z3, Z0)
        assert np.array_equal(gplan.monitor(), first)


def test_monitor_of_each_scene_in_a_batch_equals_its_single_plan():
    scenes = [scene(64, 64, 8, 1, 4, 3, 1, 2, iters=8, seed=3),
              scene(48, 36, 3, 3, 2, 1, 1, 0, iters=8, seed=4),     # no window
              scene(72, 96, 5, 2, 4, 2, 2, 3, iters=8, seed=6)]
    batch = nlpr.Batch.from_scenes(scenes, flags=nlpr.GRAPH, monitor_every=4)
    batch.solve([dev(s.Yl) for s in scenes], [dev(s.Yh) for s in scenes])
    for i, sc in enumerate(scenes):
        plan = nlpr.Plan.from_scene(sc, monitor_every=4)
        plan.solve(dev(sc.Yl), dev(sc.Yh))
        assert np.array_equal(batch.monitor(i), plan.monitor())


def test_monitor_not_enabled_and_before_first_solve():
    sc = scene(48, 36, 3, 3, 2, 1, 1, 1, iters=2)
    plan = nlpr.Plan.from_scene(sc)
    with pytest.raises(nlpr.NlprError) as e:
        plan.monitor()
    assert e.value.status == nlpr.ERR_NOT_ENABLED
    assert nlpr.Plan.from_scene(sc, monitor_every=1).monitor().shape == (0, nlpr.MON_RECORD)
