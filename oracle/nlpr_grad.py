"""FP64 reference gradient of the unrolled NLPR ADMM.

TEST INFRASTRUCTURE ONLY, like ``nlpr_oracle``: only the test suite and the benchmark's
CPU-baseline leg use it; the GPU library never calls it and shares no code with it.

The differentiated form runs T iterations of the paper's ADMM (Sec. "Optimization", the
paper's splitting, E = I) from the default start and treats the iterate X^(T) as a
function of the observations Y_l, Y_h and of the parameters lambda_2 and rho.  This module
restates that iteration in float64 torch CPU operations, literally as the numpy oracle
does (Q and Sigma for every shift of the full window W and every patch offset), so that
torch's reverse-mode automatic differentiation gives the exact gradient of any loss of
X^(T).  The weights omega of eq. (wts) are recomputed from Y_h inside, so gradients with
respect to Y_h flow both through the data term Y_h R^T and through the weights; the
thresholds lambda_2 omega / rho carry the gradients with respect to lambda_2 and rho,
which also enter the P1-update (eq. (Qh_update)) and F of eq. (Qm_update).

Only the index sets W and P are taken from ``nlpr_oracle``; every arithmetic step is
written again here so that comparing the two forwards checks both.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from .nlpr_oracle import Problem, patch_offsets

DT = torch.float64


def _shift(X: torch.Tensor, t) -> torch.Tensor:
    """Y(i) = X(i - t) on the periodic grid."""
    return torch.roll(X, shifts=(int(t[0]), int(t[1])), dims=(-2, -1))


def _filter_hat(b: np.ndarray, p: int, q: int) -> torch.Tensor:
    """DFT of the blur taps placed on the p x q grid with the centre at (0, 0)."""
    r1, r2 = b.shape[0] // 2, b.shape[1] // 2
    g = torch.zeros((p, q), dtype=DT)
    for a in range(-r1, r1 + 1):
        for c in range(-r2, r2 + 1):
            g[a % p, c % q] += float(b[a + r1, c + r2])
    return torch.fft.fft2(g)


def _D(X, tau, k):
    """D_{tau k} X (i) = X(i - k) - X(i - tau - k)."""
    return _shift(X, k) - _shift(X, (tau[0] + k[0], tau[1] + k[1]))


def _DT(Y, tau, k):
    """Adjoint of D_{tau k}: Y(j + k) - Y(j + tau + k)."""
    return _shift(Y, (-k[0], -k[1])) - _shift(Y, (-(tau[0] + k[0]), -(tau[1] + k[1])))


def weights(Yh: torch.Tensor, pr: Problem) -> torch.Tensor:
    """omega_{i tau} of eq. (wts) for every tau of the full window: [|W|][p][q]."""
    if pr.unweighted:
        return torch.ones((len(pr.window),) + tuple(Yh.shape[-2:]), dtype=DT)
    out = []
    for t in pr.window:
        e = torch.sum((Yh - _shift(Yh, t)) ** 2, dim=0)
        dist = torch.zeros_like(e)
        for k in patch_offsets(pr.K):
            dist = dist + _shift(e, k)
        out.append(torch.exp(-dist / (pr.h * pr.h)))
    return torch.stack(out)


def unrolled(Yl: torch.Tensor, Yh: torch.Tensor, lam: torch.Tensor, rho: torch.Tensor,
             pr: Problem, iters: int, init: str = "upsample", segments: int = 0) -> torch.Tensor:
    """X^(iters) of the paper's iteration (E = I), differentiable in Yl, Yh, lam, rho.

    ``segments`` > 0 changes only what reverse mode keeps in memory, not a single value:
    the iterations run in that many segments, each a recomputation checkpoint
    (``torch.utils.checkpoint``, non-reentrant) whose iterations are checkpoints in turn.
    The forward then keeps only the state entering each segment; the backward of a segment
    reruns it keeping the state entering each of its iterations, and the backward of an
    iteration reruns that iteration.  Every rerun repeats the same float64 operations on
    the same values, so the gradient is the same, bit for bit."""
    assert pr.E is None and not pr.fused
    p, q, L, d = pr.p, pr.q, pr.L, pr.d
    W, P = pr.window, patch_offsets(pr.K)
    bh = _filter_hat(pr.b, p, q)
    blur = lambda X: torch.fft.ifft2(torch.fft.fft2(X) * bh).real
    blur_T = lambda Y: torch.fft.ifft2(torch.fft.fft2(Y) * torch.conj(bh)).real
    # eq. (inv): 1 + |b^|^2 + |P| sum_{tau in W} |d^_{tau 0}|^2
    acc = torch.zeros((p, q), dtype=DT)
    for t in W:
        g = torch.zeros((p, q), dtype=DT)
        g[0, 0] += 1.0
        g[t[0] % p, t[1] % q] -= 1.0
        acc = acc + torch.abs(torch.fft.fft2(g)) ** 2
    den = 1.0 + torch.abs(bh) ** 2 + len(P) * acc
    mask = torch.zeros((p, q), dtype=DT)
    mask[::d, ::d] = 1.0
    StYl = torch.zeros((L, p, q), dtype=DT)
    StYl[:, ::d, ::d] = Yl
    R = torch.as_tensor(pr.R, dtype=DT)
    F = torch.linalg.inv(torch.eye(L, dtype=DT) + (pr.lam1 / rho) * (R @ R.T))
    YhRt = (Yh.reshape(Yh.shape[0], -1).T @ R.T)                     # n_h x L
    mu = lam * weights(Yh, pr) / rho                                  # thresholds of eq. (Qj_main)
    shape = (L, p, q)
    nwp = len(W) * len(P)

    def step(*state):
        """One iteration.  state = (P1, P2, Lam1, Lam2, Q..., Sigma...) with Q and Sigma
        listed for (tau, k) in the loop order; returns (X, new state...)."""
        P1, P2, Lam1, Lam2 = state[:4]
        Q, Sig = state[4:4 + nwp], state[4 + nwp:]
        C = blur_T(P1 + Lam1) + P2 + Lam2
        n = 0
        for t in W:
            for k in P:
                C = C + _DT(Q[n] + Sig[n], t, k)
                n += 1
        X = torch.fft.ifft2(torch.fft.fft2(C) / den).real             # eq. (inv)
        BX = blur(X)
        P1 = (mask * (rho * BX + StYl - rho * Lam1) / (1.0 + rho)
              + (1.0 - mask) * (BX - Lam1))                            # eq. (Qh_update), E = I
        A = (X - Lam2).reshape(L, -1).T + (pr.lam1 / rho) * YhRt
        P2 = (A @ F).T.reshape(shape)                                 # eq. (Qm_update)
        Qn, Sn = [], []
        n = 0
        for a, t in enumerate(W):
            for k in P:
                V = _D(X, t, k) - Sig[n]
                Qn.append(torch.sign(V) * torch.relu(torch.abs(V) - mu[a]))   # eq. (Qj_main)
                Sn.append(-(V - Qn[-1]))                                 # eq. (dualvar3_main)
                n += 1
        Lam1 = Lam1 - (BX - P1)                                       # eq. (dualvar1_main)
        Lam2 = Lam2 - (X - P2)                                        # eq. (dualvar2_main)
        return (X, P1, P2, Lam1, Lam2, *Qn, *Sn)

    if init == "upsample":
        X = Yl.repeat_interleave(d, dim=-2).repeat_interleave(d, dim=-1)
        P1, P2 = blur(X), X
    else:
        P1 = P2 = torch.zeros(shape, dtype=DT)
    zeros = lambda: torch.zeros(shape, dtype=DT)
    state = (P1, P2, zeros(), zeros(), *[zeros() for _ in range(2 * nwp)])
    if iters == 0:
        return X if init == "upsample" else torch.zeros(shape, dtype=DT)
    if segments <= 0:
        for _ in range(iters):
            X, *state = step(*state)
        return X

    from torch.utils.checkpoint import checkpoint

    def run(n_iter):
        def seg(*st):
            out = None
            for _ in range(n_iter):
                out = checkpoint(step, *st, use_reentrant=False)
                st = out[1:]
            return out
        return seg

    bounds = [iters * j // segments for j in range(segments + 1)]
    out = None
    for j in range(segments):
        n_iter = bounds[j + 1] - bounds[j]
        if n_iter == 0:
            continue
        out = checkpoint(run(n_iter), *state, use_reentrant=False)
        state = out[1:]
    return out[0]


def mse(X: torch.Tensor, Zt: torch.Tensor) -> torch.Tensor:
    return torch.mean((X - Zt) ** 2)


def gradient(Yl: np.ndarray, Yh: np.ndarray, pr: Problem, iters: int, Zt: np.ndarray,
             init: str = "upsample", segments: int = 0):
    """Loss = mean((X^(iters) - Zt)^2) and its gradient with respect to
    (Y_l, Y_h, lambda_2, rho), all float64.  ``segments``: see ``unrolled``."""
    yl = torch.tensor(np.asarray(Yl, dtype=np.float64), requires_grad=True)
    yh = torch.tensor(np.asarray(Yh, dtype=np.float64), requires_grad=True)
    lam = torch.tensor(float(pr.lam), dtype=DT, requires_grad=True)
    rho = torch.tensor(float(pr.rho), dtype=DT, requires_grad=True)
    loss = mse(unrolled(yl, yh, lam, rho, pr, iters, init, segments),
               torch.as_tensor(Zt, dtype=DT))
    loss.backward()
    return (loss.item(), yl.grad.numpy(), yh.grad.numpy(), lam.grad.item(), rho.grad.item())


def loss_at(Yl, Yh, pr: Problem, iters: int, Zt, lam: Optional[float] = None,
            rho: Optional[float] = None, init: str = "upsample") -> float:
    with torch.no_grad():
        X = unrolled(torch.as_tensor(np.asarray(Yl, dtype=np.float64)),
                     torch.as_tensor(np.asarray(Yh, dtype=np.float64)),
                     torch.tensor(float(pr.lam if lam is None else lam), dtype=DT),
                     torch.tensor(float(pr.rho if rho is None else rho), dtype=DT),
                     pr, iters, init)
        return float(mse(X, torch.as_tensor(Zt, dtype=DT)))
