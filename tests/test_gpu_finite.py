"""The device-side NaN/Inf check (NLPR_CHECK_FINITE): the iterate is checked on the device
after every 8th iteration and after the last one, without waiting; the solve reads the
flag once at the end and reports the first checked iteration that found a non-finite
value.  The fault is planted from the host: one NaN written into the Lambda2 of a stored
state, which a resumed solve (NLPR_STATE_IN) then carries into every pixel of X."""
import numpy as np
import pytest
import torch

import synth
from paper_2210_04184_amd import nlpr

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_check_leaves_a_clean_solve_unchanged():
    spec = synth.small_spec(p=64, q=96, L=6, Lh=2, d=4, K=1, Sw=1, iters=20, seed=51)
    sc = synth.make_scene(spec)
    print("[finite] 64x96x6, 20 iterations, clean", flush=True)
    a = nlpr.Plan.from_scene(sc, flags=nlpr.CHECK_FINITE)
    b = nlpr.Plan.from_scene(sc)
    try:
        Za, _ = a.solve(dev(sc.Yl), dev(sc.Yh))
        Zb, _ = b.solve(dev(sc.Yl), dev(sc.Yh))
        torch.cuda.synchronize()
        assert a.nonfinite_iteration() == -1
        assert torch.equal(Za, Zb)
        with pytest.raises(nlpr.NlprError) as e:
            b.nonfinite_iteration()
        assert e.value.status == nlpr.ERR_NOT_ENABLED
    finally:
        a.close()
        b.close()


@pytest.mark.parametrize("iters,first", [(20, 8), (5, 5), (16, 8)])
def test_first_bad_iteration_of_a_resumed_solve(iters, first):
    spec = synth.small_spec(p=64, q=96, L=6, Lh=2, d=4, K=1, Sw=1, iters=10, seed=52)
    sc = synth.make_scene(spec)
    print(f"[finite] 64x96x6: 10 iterations, NaN planted in Lambda2, {iters} resumed", flush=True)
    start = nlpr.Plan.from_scene(sc, flags=nlpr.CHECK_FINITE)
    resume = nlpr.Plan.from_scene(sc, flags=nlpr.CHECK_FINITE | nlpr.STATE_IN, iters=iters)
    try:
        Yl, Yh = dev(sc.Yl), dev(sc.Yh)
        Z, ws = start.solve(Yl, Yh)
        assert start.nonfinite_iteration() == -1
        lam2 = resume.region_view(ws, nlpr.REGION_LAMBDA2)
        lam2[3 * spec.p * spec.q + 17 * spec.q + 40] = float("nan")
        with pytest.raises(nlpr.NlprError) as e:
            resume.solve(Yl, Yh, Z=Z, ws=ws)
        assert e.value.status == nlpr.ERR_NUMERICAL
        assert f"after iteration {first}" in str(e.value)
        assert resume.nonfinite_iteration() == first
        assert not bool(torch.isfinite(Z).any())
    finally:
        start.close()
        resume.close()
