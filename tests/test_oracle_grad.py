"""Pins of the FP64 reference gradient (``oracle.nlpr_grad``).

Its forward must equal the numpy oracle's iterate, and its reverse-mode gradient must
equal central finite differences of the same float64 loss: for lambda_2 and rho
directly, for Y_l and Y_h along random directions.  Finite differences use a relative
step of 1e-6, far below the distance of any iterate from a kink of the soft threshold on
these random inputs.
"""
import numpy as np
import pytest
import torch

from oracle import nlpr_grad as g
from oracle import nlpr_oracle as o
from test_oracle_pins import tiny_problem


def problem(seed=0, **kw):
    args = dict(p=8, q=12, L=3, Lh=2, d=2, r=1, K=1, S=1, lam=0.08, rho=0.4, lam1=0.9, h=0.8)
    args.update(kw)
    return tiny_problem(seed=seed, **args)


@pytest.mark.parametrize("kw", [{}, dict(local=True), dict(unweighted=True), dict(K=0, S=2)])
def test_forward_equals_numpy_oracle(kw):
    pr, Yl, Yh = problem(**kw)
    want = o.solve(Yl, Yh, pr, 4).X
    with torch.no_grad():
        got = g.unrolled(torch.as_tensor(Yl), torch.as_tensor(Yh),
                         torch.tensor(pr.lam, dtype=torch.float64),
                         torch.tensor(pr.rho, dtype=torch.float64), pr, 4).numpy()
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


@pytest.mark.parametrize("kw", [{}, dict(local=True), dict(unweighted=True)])
def test_gradient_equals_central_differences(kw):
    pr, Yl, Yh = problem(seed=2, **kw)
    T = 4
    rng = np.random.default_rng(9)
    Zt = rng.uniform(0, 1, (pr.L, pr.p, pr.q))
    loss, gYl, gYh, glam, grho = g.gradient(Yl, Yh, pr, T, Zt)
    assert loss == pytest.approx(g.loss_at(Yl, Yh, pr, T, Zt), rel=1e-14)
    f = lambda **kw_: g.loss_at(kw_.get("Yl", Yl), kw_.get("Yh", Yh), pr, T, Zt,
                                lam=kw_.get("lam"), rho=kw_.get("rho"))
    for name, val, grad in (("lam", pr.lam, glam), ("rho", pr.rho, grho)):
        h = 1e-6 * val
        fd = (f(**{name: val + h}) - f(**{name: val - h})) / (2 * h)
        assert grad == pytest.approx(fd, rel=1e-6, abs=1e-12), name
    for name, arr, grad in (("Yl", Yl, gYl), ("Yh", Yh, gYh)):
        v = rng.standard_normal(arr.shape)
        h = 1e-6
        fd = (f(**{name: arr + h * v}) - f(**{name: arr - h * v})) / (2 * h)
        assert float(np.sum(grad * v)) == pytest.approx(fd, rel=1e-6), name
    if kw.get("unweighted"):
        return
    # the weights carry part of the Y_h gradient: it changes when they are frozen
    assert np.linalg.norm(gYh) > 0


def test_gradient_from_the_zero_start():
    # with init = "zero" Y_l enters only through the P1-update on sampled pixels
    pr, Yl, Yh = problem(seed=4)
    Zt = np.zeros((pr.L, pr.p, pr.q))
    _, gYl, _, _, _ = g.gradient(Yl, Yh, pr, 3, Zt, init="zero")
    v = np.random.default_rng(1).standard_normal(Yl.shape)
    fd = (g.loss_at(Yl + 1e-6 * v, Yh, pr, 3, Zt, init="zero")
          - g.loss_at(Yl - 1e-6 * v, Yh, pr, 3, Zt, init="zero")) / 2e-6
    assert float(np.sum(gYl * v)) == pytest.approx(fd, rel=1e-6)


@pytest.mark.parametrize("segments", [1, 2, 3])
def test_recomputation_checkpoints_leave_every_bit(segments):
    """Segments of recomputation change what reverse mode keeps, not the arithmetic."""
    pr, Yl, Yh = problem(seed=6)
    Zt = np.random.default_rng(3).uniform(0, 1, (pr.L, pr.p, pr.q))
    a = g.gradient(Yl, Yh, pr, 5, Zt)
    b = g.gradient(Yl, Yh, pr, 5, Zt, segments=segments)
    assert a[0] == b[0] and a[3] == b[3] and a[4] == b[4]
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])
