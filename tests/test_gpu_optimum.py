"""The GPU solve against the mathematics rather than against the oracle's iterates.

Theorem 1 of the paper: from any start and for any rho > 0 the ADMM iterates reach a
minimiser of eq. (ouroptim).  On a tiny problem the optimal value is computed independently,
by a Chambolle-Pock primal-dual solver on dense matrices of S, B, R and every D_{tau k}
(the same construction that pins the oracle in test_oracle_pins).  Several minimisers may
exist (the l1 term is not strictly convex and S B, R are rank-deficient), so objective values
are compared, not iterates.

Tolerances.  The GPU iterates are FP32: after tens of thousands of iterations the objective
of X^T (evaluated in FP64) lies within 1e-5 relative of the optimum (measured: about 1e-7).
The FP32 iteration is non-expansive, so rounding does not accumulate: after 1000 iterations
X^T still meets the 1e-4 relative-RMSE bar against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

from oracle import nlpr_oracle as o
from paper_2210_04184_amd import nlpr
from test_oracle_pins import _dense_objective, _dense_problem, _pdhg, tiny_problem, vec

pytestmark = pytest.mark.gpu

# at the optimum 46 % ("mild") and 84 % ("strong") of the weighted differences D_{tau k} X are
# zero: both regimes of the shrinkage are active (a larger lambda_2 makes every band constant)
PROBLEMS = {
    "mild": dict(lam=0.02, h=0.7, seed=0),
    "strong": dict(lam=0.04, h=0.7, seed=1),
}


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def problem(name):
    """8 x 8 image, 2 bands, 1 guide band, d = 2, 3 x 3 blur, patch 3 x 3, window 3 x 3;
    inputs, blur and R rounded to FP32 once and shared by every solver."""
    pr, Yl, Yh = tiny_problem(p=8, q=8, L=2, Lh=1, d=2, K=1, S=1, **PROBLEMS[name])
    pr.b, pr.R = f32(pr.b), f32(pr.R)
    return pr, f32(Yl), f32(Yh)


_OPT = {}


def optimum(name):
    if name not in _OPT:
        pr, Yl, Yh = problem(name)
        H, bb, c0, G, w = _dense_problem(pr, Yl, Yh)
        x = _pdhg(H, bb, G, w, 4000)     # converged: 16000 iterations give the same value
        _OPT[name] = (_dense_objective(x, H, bb, c0, G, w), (H, bb, c0, G, w))
    return _OPT[name]


def gpu_solve(pr, Yl, Yh, iters, flags=0):
    plan = nlpr.Plan(p=pr.p, q=pr.q, L=pr.L, Lh=pr.R.shape[1], d=pr.d, blur=pr.b, R=pr.R,
                     K=pr.K, Sw=pr.S, iters=iters, lam=pr.lam, rho=pr.rho, h=pr.h,
                     lam1=pr.lam1, E=pr.E, flags=flags)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    Z, _ = plan.solve(dev(Yl), dev(Yh))
    torch.cuda.synchronize()
    return Z.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("name", list(PROBLEMS))
@pytest.mark.parametrize("rho,iters", [(0.3, 20000), (1.0, 40000)])
def test_gpu_solve_reaches_the_optimum_of_an_independent_solver(name, rho, iters):
    f_opt, dense = optimum(name)
    pr, Yl, Yh = problem(name)
    pr.rho = rho
    X = gpu_solve(pr, Yl, Yh, iters)
    f = _dense_objective(vec(X).T.ravel(), *dense)
    print(f"[optimum {name} rho={rho}] f_gpu={f!r} f_opt={f_opt!r} rel={(f - f_opt) / f_opt:.2e}",
          flush=True)
    assert f == pytest.approx(f_opt, rel=1e-5)


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_unsplit_x_update_reaches_the_same_optimum(name):
    """The un-split X-update (S B inside the X-subproblem) follows other iterates but, by the
    same theorem, reaches the same optimal value."""
    f_opt, dense = optimum(name)
    pr, Yl, Yh = problem(name)
    X = gpu_solve(pr, Yl, Yh, 20000, flags=nlpr.FUSED_S)
    f = _dense_objective(vec(X).T.ravel(), *dense)
    assert f == pytest.approx(f_opt, rel=1e-5)


def test_long_run_stays_within_the_bar_of_the_fp64_oracle():
    pr, Yl, Yh = problem("strong")
    X = gpu_solve(pr, Yl, Yh, 1000)
    ref = o.solve(Yl, Yh, pr, 1000).X
    assert np.linalg.norm(X - ref) / np.linalg.norm(ref) <= 1e-4


# the other regularisers and the subspace form, each with part of the differences zero at the
# optimum (68 %, 52 %, 66 %); the dense solve is converged to 1e-10 at 16 000 iterations
VARIANTS = {
    "subspace": (dict(L=3, Lh=1, lam=0.02, h=0.7, Ls=2, seed=0), 0),
    "unweighted": (dict(L=2, Lh=1, lam=0.002, h=0.7, unweighted=True, seed=0), nlpr.UNWEIGHTED),
    "local": (dict(L=2, Lh=1, lam=0.05, h=0.7, local=True, seed=1), nlpr.LOCAL_WINDOW),
}


@pytest.mark.parametrize("name", list(VARIANTS))
def test_variants_reach_the_optimum_of_an_independent_solver(name):
    kw, flags = VARIANTS[name]
    pr, Yl, Yh = tiny_problem(p=8, q=8, d=2, K=1, S=1, rho=0.3, **kw)
    pr.b, pr.R, Yl, Yh = f32(pr.b), f32(pr.R), f32(Yl), f32(Yh)
    if pr.E is not None:
        pr.E = f32(pr.E)
    H, bb, c0, G, w = _dense_problem(pr, Yl, Yh)
    f_opt = _dense_objective(_pdhg(H, bb, G, w, 16000), H, bb, c0, G, w)
    Z = gpu_solve(pr, Yl, Yh, 20000, flags=flags)
    # the objective is a function of the coefficient image X (Z = X E, E of full row rank)
    X = vec(Z) if pr.E is None else vec(Z) @ np.linalg.pinv(pr.E)
    f = _dense_objective(X.T.ravel(), H, bb, c0, G, w)
    print(f"[optimum {name}] rel={(f - f_opt) / f_opt:.2e}", flush=True)
    assert f == pytest.approx(f_opt, rel=1e-5)
