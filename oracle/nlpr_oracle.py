"""FP64 CPU oracle of the guided nonlocal patch-regularised (NLPR) fusion ADMM.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg import this module.  The GPU library never calls it, and it shares no
code with the GPU path.

Paper: Unni V. S., P. Nair, K. N. Chaudhury, "Guided Nonlocal Patch Regularization and
Efficient Filtering-Based Inversion for Multiband Fusion" (arXiv 2210.04184).

The oracle is the paper's *literal* iteration: it keeps a latent variable Q_{tau k} and a
dual Sigma_{tau k} for every shift tau in the full search window W = [-S, S]^2
(tau = 0 included) and every patch offset k in P = [-K, K]^2, and performs the updates
of Sec. "Optimization" in the paper's order:

    X-update   eq. (x_linear_system_main) solved in Fourier by eq. (inv)
    P1-update  eq. (Qh_update)
    P2-update  eq. (Qm_update)
    Q-update   eq. (Qj_main)                     (soft thresholding)
    duals      eqs. (dualvar1_main) - (dualvar3_main)

It is plain numpy: arrays are float64, circular shifts are ``np.roll`` and the FFT is
``numpy.fft``.  No blocking, fusion or reordering beyond the definitions.

Notation and storage.  The paper writes an image with L bands as a matrix
X in R^{n_h x L} (one row per pixel).  Here images are stored planar,
``X[c][i1][i2]`` (band, row, col), and converted to the paper's matrix form by
``to_mat`` whenever a formula multiplies on the band axis.

Readings of points the paper leaves open:
  * The subspace basis E (L_s x L, Z = X E) is optional; without it E = I and X is Z.
  * With a basis, the default start is the least-squares coefficient image of the
    upsampled Y_l: X0 = up(Y_l) E^T (E E^T)^{-1}.
  * The one "lambda" of a workload is lambda_2; lambda_1 defaults to 1.
  * The Q-update threshold is lambda_2 * omega / rho, as printed in eq. (Qj_main);
    the objective is ell(X) + lambda_2 * phi(X) as in eq. (mainoptim).
  * K is the patch radius (P = [-K, K]^2) and S the search radius (W = [-S, S]^2).
  * The blur kernel is centred at (0, 0) and applied circularly; S keeps the pixels
    (d*m1, d*m2).
  * Initial values (the paper names them but does not give them): X0 is the
    nearest-neighbour upsample of Y_l, P1 = B X0, P2 = X0, Q = Sigma = Lambda = 0;
    ``init="zero"`` starts every variable at 0.
  * The patch distance of eq. (wts) is the plain sum of squared differences over all
    (2K+1)^2 L_h entries of the patch, without normalisation.
  * Besides the paper's splitting, ``Problem.fused`` selects a splitting without P1 that
    keeps S B in the X-subproblem (the aliasing-group solve below); E = I there, and its
    default start is that of the paper's splitting without P1 and Lambda1.
"""
from __future__ import annotations

import dataclasses
from concurrent.futures import ThreadPoolExecutor
from typing import Callable, Iterator, List, Optional, Sequence, Tuple

import numpy as np

Offset = Tuple[int, int]


# ----------------------------------------------------------------------------- sets
def search_window(S: int, local: bool = False) -> List[Offset]:
    """W = [-S, S]^2 (Sec. "Definition").  ``local`` gives the 4-neighbour window
    {0, +-e1, +-e2} of the local pixel regulariser (ablation case C5)."""
    if local:
        return [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
    return [(a, b) for a in range(-S, S + 1) for b in range(-S, S + 1)]


def patch_offsets(K: int) -> List[Offset]:
    """P = [-K, K]^2, the offsets k of a (2K+1) x (2K+1) patch (Sec. "Definition")."""
    return [(a, b) for a in range(-K, K + 1) for b in range(-K, K + 1)]


# ----------------------------------------------------------------------- operators
def shift(X: np.ndarray, t: Offset) -> np.ndarray:
    """Circular shift on the periodic domain: returns Y with Y(i) = X(i - t), indices
    taken mod (p, q) (Sec. "Definition")."""
    return np.roll(X, shift=(t[0], t[1]), axis=(-2, -1))


def to_mat(X: np.ndarray) -> np.ndarray:
    """Planar [L][p][q] -> the paper's n_h x L matrix (row = pixel, column = band)."""
    return X.reshape(X.shape[0], -1).T


def from_mat(M: np.ndarray, p: int, q: int) -> np.ndarray:
    return np.ascontiguousarray(M.T).reshape(M.shape[1], p, q)


def blur_filter_grid(b: np.ndarray, p: int, q: int) -> np.ndarray:
    """The blur filter b placed on the periodic p x q grid with its centre at (0, 0)."""
    r1, r2 = b.shape[0] // 2, b.shape[1] // 2
    g = np.zeros((p, q))
    for a in range(-r1, r1 + 1):
        for c in range(-r2, r2 + 1):
            g[a % p, c % q] += b[a + r1, c + r2]
    return g


def blur(X: np.ndarray, b: np.ndarray) -> np.ndarray:
    """B X: circular convolution (b * X_c)(i) = sum_m b(m) X_c(i - m) for every band,
    computed as the product of DFTs (eq. (model); B is a circular blur)."""
    p, q = X.shape[-2:]
    bh = np.fft.fft2(blur_filter_grid(b, p, q))
    return np.fft.ifft2(np.fft.fft2(X) * bh).real


def blur_T(Y: np.ndarray, b: np.ndarray) -> np.ndarray:
    """B^T Y: the adjoint of ``blur`` (correlation, filter conj(b^))."""
    p, q = Y.shape[-2:]
    bh = np.fft.fft2(blur_filter_grid(b, p, q))
    return np.fft.ifft2(np.fft.fft2(Y) * np.conj(bh)).real


def decimate(X: np.ndarray, d: int) -> np.ndarray:
    """S X: keep pixels (d*m1, d*m2)."""
    return X[..., ::d, ::d]


def decimate_T(Y: np.ndarray, d: int, p: int, q: int) -> np.ndarray:
    """S^T Y: place the low-resolution pixels at (d*m1, d*m2), zero elsewhere."""
    out = np.zeros(Y.shape[:-2] + (p, q))
    out[..., ::d, ::d] = Y
    return out


def sampling_mask(p: int, q: int, d: int) -> np.ndarray:
    """Diagonal of S^T S: 1 on the sampled pixels, 0 elsewhere (eq. (maskprop))."""
    m = np.zeros((p, q))
    m[::d, ::d] = 1.0
    return m


def spectral(X: np.ndarray, R: np.ndarray) -> np.ndarray:
    """X R in the paper's matrix form (n_h x L times L x L_h), returned planar."""
    p, q = X.shape[-2:]
    return from_mat(to_mat(X) @ R, p, q)


def D(X: np.ndarray, tau: Offset, k: Offset) -> np.ndarray:
    """Difference operator of eq. (differencemat): D_{tau k} X(i, c) = X_c(i - k) - X_c(i - tau - k)."""
    return shift(X, k) - shift(X, (tau[0] + k[0], tau[1] + k[1]))


def D_T(Y: np.ndarray, tau: Offset, k: Offset) -> np.ndarray:
    """Adjoint of D_{tau k}: (D^T Y)(j) = Y(j + k) - Y(j + tau + k)."""
    return shift(Y, (-k[0], -k[1])) - shift(Y, (-(tau[0] + k[0]), -(tau[1] + k[1])))


def soft_threshold(x: np.ndarray, mu) -> np.ndarray:
    """S(x, mu) = sign(x) max(|x| - mu, 0), componentwise (after eq. (Qj_main))."""
    return np.sign(x) * np.maximum(np.abs(x) - mu, 0.0)


# ------------------------------------------------------------------------- weights
def patch_distance(Yh: np.ndarray, tau: Offset, K: int) -> np.ndarray:
    """||P_{i tau}(Y_h)||_2^2 for every pixel i: the sum over (k, c) in Lambda of
    (Y_c(i - k) - Y_c(i - tau - k))^2 (Sec. "Definition").  The squared differences of
    the band images are summed over c first, then gathered over the patch offsets k."""
    e = np.sum((Yh - shift(Yh, tau)) ** 2, axis=0)     # e(j) = sum_c (Y_c(j) - Y_c(j - tau))^2
    out = np.zeros_like(e)
    for k in patch_offsets(K):
        out += shift(e, k)                              # e(i - k)
    return out


def weights(Yh: np.ndarray, window: Sequence[Offset], K: int, h: float,
            unweighted: bool = False) -> np.ndarray:
    """omega_{i tau} of eq. (wts) for every tau in ``window``: array [|W|][p][q]."""
    p, q = Yh.shape[-2:]
    if unweighted:
        return np.ones((len(window), p, q))
    return np.stack([np.exp(-patch_distance(Yh, t, K) / (h * h)) for t in window])


# -------------------------------------------------------------------- X-update solve
def denominator(p: int, q: int, b: np.ndarray, window: Sequence[Offset], K: int) -> np.ndarray:
    """1 + |b^(w)|^2 + |P| sum_{tau in W} |d^_{tau 0}(w)|^2 of eq. (inv), where d_{tau 0}
    is +1 at 0 and -1 at tau on the periodic grid (Sec. "Patch variation using
    convolutions")."""
    bh = np.fft.fft2(blur_filter_grid(b, p, q))
    acc = np.zeros((p, q))
    for t in window:
        dgrid = np.zeros((p, q))
        dgrid[0, 0] += 1.0
        dgrid[t[0] % p, t[1] % q] -= 1.0
        acc += np.abs(np.fft.fft2(dgrid)) ** 2
    return 1.0 + np.abs(bh) ** 2 + len(patch_offsets(K)) * acc


def x_update(C: np.ndarray, den: np.ndarray) -> np.ndarray:
    """Solve (I + B^T B + sum D^T D) X = C band by band: X_c = IDFT(DFT(C_c) / den)
    (eqs. (xupdateoper), (inv))."""
    return np.fft.ifft2(np.fft.fft2(C) / den).real


# ------------------------------------------ X-update with S inside the system (fused-S)
# A variant of the splitting of eq. (fusionoptim) without P1: the data term
# 1/2 ||Y_l - S B X||^2 stays in the X-subproblem, whose normal equation becomes
#   (I + sum_{tau, k} D^T D + B^T S^T S B / rho) X = B^T S^T Y_l / rho + P2 + Lambda2
#                                                   + sum_{tau, k} D^T (Q + Sigma).
# It has the same minimiser as the paper's splitting (both are ADMM on a split of the
# same objective) and different iterates.  The first two terms are diagonal in Fourier
# (eqs. (xupdateoper), (inv) without the blur); S^T S is the sampling mask, which in
# Fourier averages each frequency with its d^2 - 1 aliases w + (m1 p/d, m2 q/d).
def fused_denominator(p: int, q: int, window: Sequence[Offset], K: int) -> np.ndarray:
    """a(w) = 1 + |P| sum_{tau in W} |d^_{tau 0}(w)|^2: the denominator of eq. (inv)
    without the blur term."""
    return denominator(p, q, np.zeros((1, 1)), window, K)


def aliasing_groups(p: int, q: int, d: int) -> np.ndarray:
    """Index arrays [groups][d^2] (rows, cols) of the frequencies the mask S^T S couples:
    (w1 + m1 p/d, w2 + m2 q/d) for m1, m2 in [0, d), one group per (w1, w2) in
    [0, p/d) x [0, q/d)."""
    pd, qd = p // d, q // d
    w1, w2 = np.meshgrid(np.arange(pd), np.arange(qd), indexing="ij")
    m1, m2 = np.meshgrid(np.arange(d), np.arange(d), indexing="ij")
    rows = w1.reshape(-1, 1) + pd * m1.reshape(1, -1)
    cols = w2.reshape(-1, 1) + qd * m2.reshape(1, -1)
    return rows, cols


def x_update_fused(C: np.ndarray, pr: Problem, a: np.ndarray) -> np.ndarray:
    """Solve (I + sum D^T D + B^T S^T S B / rho) X = C band by band.  In Fourier the
    system is a(w) x^(w) + conj(b^(w)) / (rho d^2) sum_{w' ~ w} b^(w') x^(w'), with w' over
    the aliasing group of w: one dense d^2 x d^2 complex system per group, solved
    directly."""
    p, q, d = pr.p, pr.q, pr.d
    bh = np.fft.fft2(blur_filter_grid(pr.b, p, q))
    rows, cols = aliasing_groups(p, q, d)
    bv = bh[rows, cols]                                             # [G][d^2]
    A = np.zeros(bv.shape + (bv.shape[1],), dtype=complex)
    A[:, np.arange(d * d), np.arange(d * d)] = a[rows, cols]
    A += np.conj(bv)[:, :, None] * bv[:, None, :] / (pr.rho * d * d)
    Ch = np.fft.fft2(C)                                             # [L][p][q]
    rhs = np.moveaxis(Ch[:, rows, cols], 0, -1)                     # [G][d^2][L]
    sol = np.linalg.solve(A, rhs)
    Xh = np.empty_like(Ch)
    Xh[:, rows, cols] = np.moveaxis(sol, -1, 0)
    return np.fft.ifft2(Xh).real


# ----------------------------------------------------------------------- problem
@dataclasses.dataclass
class Problem:
    """Everything the iteration needs besides the observations."""

    p: int
    q: int
    L: int
    d: int
    b: np.ndarray           # blur taps [2r+1][2r+1]
    R: np.ndarray           # spectral response [L][Lh]
    K: int
    S: int
    lam: float              # lambda_2
    rho: float
    h: float
    lam1: float = 1.0       # lambda_1
    unweighted: bool = False
    local: bool = False
    E: Optional[np.ndarray] = None   # subspace basis [Ls][L] (Z = X E); None means E = I
    fused: bool = False     # keep S B inside the X-subproblem (no P1 split); E = I only

    @property
    def Ebasis(self) -> np.ndarray:
        return np.eye(self.L) if self.E is None else self.E

    @property
    def Ls(self) -> int:
        """Bands of X (rows of E)."""
        return self.L if self.E is None else self.E.shape[0]

    @classmethod
    def from_scene(cls, scene, **kw) -> "Problem":
        s = scene.spec
        args = dict(p=s.p, q=s.q, L=s.L, d=s.d, b=scene.blur.astype(np.float64),
                    R=scene.R.astype(np.float64), K=s.K, S=s.Sw, lam=s.lam, rho=s.rho,
                    h=scene.h, lam1=s.lam1)
        args.update(kw)
        return cls(**args)

    @property
    def window(self) -> List[Offset]:
        return search_window(self.S, self.local)

    @property
    def patch(self) -> List[Offset]:
        return patch_offsets(self.K)


def upsample_nn(Yl: np.ndarray, d: int) -> np.ndarray:
    """Nearest-neighbour upsample: X0(i) = Y_l(floor(i1/d), floor(i2/d))."""
    return np.repeat(np.repeat(Yl, d, axis=-2), d, axis=-1)


def p1_update(BX: np.ndarray, Lam1: np.ndarray, Yl: np.ndarray, pr: Problem) -> np.ndarray:
    """eq. (Qh_update):
    P1 = S^T S (rho B X + S^T Y_l E^T - rho Lambda1)(E E^T + rho I)^{-1} + (I - S^T S)(B X - Lambda1)."""
    M = to_mat(sampling_mask(pr.p, pr.q, pr.d)[None])            # n_h x 1 diagonal of S^T S
    E = pr.Ebasis
    inv = np.linalg.inv(E @ E.T + pr.rho * np.eye(pr.Ls))
    StYl = decimate_T(Yl, pr.d, pr.p, pr.q)
    sampled = (pr.rho * to_mat(BX) + to_mat(StYl) @ E.T - pr.rho * to_mat(Lam1)) @ inv
    rest = to_mat(BX) - to_mat(Lam1)
    return from_mat(M * sampled + (1.0 - M) * rest, pr.p, pr.q)


def p2_matrix(pr: Problem) -> np.ndarray:
    """F = (I + lambda1/rho E R R^T E^T)^{-1}, L_s x L_s (after eq. (Qm_update))."""
    E = pr.Ebasis
    return np.linalg.inv(np.eye(pr.Ls) + (pr.lam1 / pr.rho) * (E @ pr.R @ pr.R.T @ E.T))


def p2_update(X: np.ndarray, Lam2: np.ndarray, Yh: np.ndarray, pr: Problem,
              F: Optional[np.ndarray] = None) -> np.ndarray:
    """eq. (Qm_update): P2 = (-Lambda2 + X + lambda1/rho Y_h R^T E^T) F."""
    if F is None:
        F = p2_matrix(pr)
    A = -to_mat(Lam2) + to_mat(X) + (pr.lam1 / pr.rho) * (to_mat(Yh) @ pr.R.T @ pr.Ebasis.T)
    return from_mat(A @ F, pr.p, pr.q)


# --------------------------------------------------------------------- objective
def regulariser(X: np.ndarray, omega: np.ndarray, window: Sequence[Offset],
                K: int) -> float:
    """phi(X) in its filter form eq. (regfilt1):
    sum_i sum_c sum_{tau in W} sum_{k in P} omega_{i tau} |D_{tau k} X(i, c)|."""
    tot = 0.0
    for n, t in enumerate(window):
        for k in patch_offsets(K):
            tot += float(np.sum(omega[n][None] * np.abs(D(X, t, k))))
    return tot


def objective_terms(X: np.ndarray, Yl: np.ndarray, Yh: np.ndarray, pr: Problem,
                    omega: Optional[np.ndarray] = None) -> Tuple[float, float, float]:
    """The three terms of eq. (mainoptim): 1/2 ||Y_l - S B Z||^2, lambda1/2 ||Y_h - Z R||^2
    and lambda2 phi(X), with Z = X E."""
    if omega is None:
        omega = weights(Yh, pr.window, pr.K, pr.h, pr.unweighted)
    Z = compose(X, pr)
    r1 = Yl - decimate(blur(Z, pr.b), pr.d)
    r2 = Yh - spectral(Z, pr.R)
    return (0.5 * float(np.sum(r1 * r1)), 0.5 * pr.lam1 * float(np.sum(r2 * r2)),
            pr.lam * regulariser(X, omega, pr.window, pr.K))


def objective(X: np.ndarray, Yl: np.ndarray, Yh: np.ndarray, pr: Problem,
              omega: Optional[np.ndarray] = None) -> float:
    """ell(X) + lambda2 phi(X), eq. (mainoptim): the data terms act on Z = X E."""
    return float(sum(objective_terms(X, Yl, Yh, pr, omega)))


# ------------------------------------------------------------------------- ADMM
@dataclasses.dataclass
class State:
    """ADMM variables: primal P1, P2, Q and duals Lambda1, Lambda2, Sigma.
    Q and Sigma are [|W|][|P|][L][p][q]."""

    P1: np.ndarray
    P2: np.ndarray
    Q: np.ndarray
    Lam1: np.ndarray
    Lam2: np.ndarray
    Sig: np.ndarray


def compose(X: np.ndarray, pr: Problem) -> np.ndarray:
    """Z = X E (the low-rank representation); X itself when E = I."""
    if pr.E is None:
        return X
    return from_mat(to_mat(X) @ pr.E, pr.p, pr.q)


def initial_state(Yl: np.ndarray, pr: Problem, init: str = "upsample") -> Tuple[np.ndarray, State]:
    shape = (pr.Ls, pr.p, pr.q)
    nw, npch = len(pr.window), len(pr.patch)
    if init == "upsample":
        X0 = upsample_nn(Yl.astype(np.float64), pr.d)
        if pr.E is not None:
            E = pr.E
            X0 = from_mat(to_mat(X0) @ E.T @ np.linalg.inv(E @ E.T), pr.p, pr.q)
        P1, P2 = blur(X0, pr.b), X0.copy()
        if pr.fused:                   # no P1 in the fused-S splitting
            P1 = np.zeros(shape)
    elif init == "zero":
        X0 = np.zeros(shape)
        P1, P2 = np.zeros(shape), np.zeros(shape)
    else:
        raise ValueError(init)
    z = np.zeros(shape)
    st = State(P1=P1, P2=P2, Q=np.zeros((nw, npch) + shape), Lam1=z.copy(), Lam2=z.copy(),
               Sig=np.zeros((nw, npch) + shape))
    return X0, st


# The (tau, k) loops below may run on a thread pool (``workers`` > 1).  That changes no
# arithmetic: every (tau, k) term is computed by the same numpy calls, the Q and Sigma
# updates write disjoint slices, and the terms of the sum over (tau, k) are still added
# to C one at a time in the serial loop order, so the result is bit-identical to one worker.
def _in_order(pool: Optional[ThreadPoolExecutor], fn: Callable, items: Sequence) -> Iterator:
    """fn(x) for every x of ``items``, yielded in the order of ``items``.  With a pool, a
    few items per worker are computed at a time, so at most that many results are held."""
    if pool is None:
        for x in items:
            yield fn(x)
        return
    step = 4 * pool._max_workers
    for s in range(0, len(items), step):
        yield from pool.map(fn, items[s:s + step])


def _pairs(pr: Problem) -> List[Tuple[int, Offset, int, Offset]]:
    """(n, tau, m, k) for tau = window[n], k = patch[m], in the loop order of the sums."""
    return [(n, t, m, k) for n, t in enumerate(pr.window) for m, k in enumerate(pr.patch)]


def rhs(st: State, pr: Problem, pool: Optional[ThreadPoolExecutor] = None) -> np.ndarray:
    """C = B^T(P1 + Lambda1) + P2 + Lambda2 + sum_tau sum_k D_{tau k}^T (Q_{tau k} + Sigma_{tau k})
    (after eq. (x_linear_system_main))."""
    C = blur_T(st.P1 + st.Lam1, pr.b) + st.P2 + st.Lam2
    term = lambda a: D_T(st.Q[a[0], a[2]] + st.Sig[a[0], a[2]], a[1], a[3])
    for T in _in_order(pool, term, _pairs(pr)):
        C += T
    return C


def admm_step(st: State, Yl: np.ndarray, Yh: np.ndarray, pr: Problem, den: np.ndarray,
              mu: np.ndarray, F: np.ndarray,
              pool: Optional[ThreadPoolExecutor] = None) -> Tuple[np.ndarray, State]:
    """One ADMM iteration t -> t+1 in the paper's order.  ``mu`` = lambda2 omega / rho."""
    X = x_update(rhs(st, pr, pool), den)                             # eq. (inv)
    BX = blur(X, pr.b)
    P1 = p1_update(BX, st.Lam1, Yl, pr)                              # eq. (Qh_update)
    P2 = p2_update(X, st.Lam2, Yh, pr, F)                            # eq. (Qm_update)
    Q = np.empty_like(st.Q)
    Sig = np.empty_like(st.Sig)

    def q_sigma(a):
        n, t, m, k = a
        DX = D(X, t, k)
        Q[n, m] = soft_threshold(DX - st.Sig[n, m], mu[n][None])      # eq. (Qj_main)
        Sig[n, m] = st.Sig[n, m] - (DX - Q[n, m])                     # eq. (dualvar3_main)

    for _ in _in_order(pool, q_sigma, _pairs(pr)):
        pass
    Lam1 = st.Lam1 - (BX - P1)                                       # eq. (dualvar1_main)
    Lam2 = st.Lam2 - (X - P2)                                        # eq. (dualvar2_main)
    return X, State(P1=P1, P2=P2, Q=Q, Lam1=Lam1, Lam2=Lam2, Sig=Sig)


def admm_step_fused(st: State, Yl: np.ndarray, Yh: np.ndarray, pr: Problem, a: np.ndarray,
                    C0: np.ndarray, mu: np.ndarray, F: np.ndarray) -> Tuple[np.ndarray, State]:
    """One iteration of the fused-S variant: the X-update solves the system above with
    right-hand side C0 + P2 + Lambda2 + sum D^T (Q + Sigma), C0 = B^T S^T Y_l / rho; then
    P2, Q, Lambda2 and Sigma as in the paper's iteration.  P1 and Lambda1 stay 0."""
    C = C0 + st.P2 + st.Lam2
    for n, t in enumerate(pr.window):
        for m, k in enumerate(pr.patch):
            C += D_T(st.Q[n, m] + st.Sig[n, m], t, k)
    X = x_update_fused(C, pr, a)
    P2 = p2_update(X, st.Lam2, Yh, pr, F)                            # eq. (Qm_update)
    Q = np.empty_like(st.Q)
    Sig = np.empty_like(st.Sig)
    for n, t in enumerate(pr.window):
        for m, k in enumerate(pr.patch):
            DX = D(X, t, k)
            Q[n, m] = soft_threshold(DX - st.Sig[n, m], mu[n][None])  # eq. (Qj_main)
            Sig[n, m] = st.Sig[n, m] - (DX - Q[n, m])                 # eq. (dualvar3_main)
    Lam2 = st.Lam2 - (X - P2)                                        # eq. (dualvar2_main)
    return X, State(P1=st.P1, P2=P2, Q=Q, Lam1=st.Lam1, Lam2=Lam2, Sig=Sig)


def fixed_point_residual(a: State, b: State, rho: float) -> float:
    """rho (||V^{t+1} - V^t||^2 + ||U^{t+1} - U^t||^2) with V = (P1, P2, Q) and
    U = (Lambda1, Lambda2, Sigma), the grouping of the Appendix (eqs. (Vdef2), (Udef))."""
    s = 0.0
    for f in ("P1", "P2", "Q", "Lam1", "Lam2", "Sig"):
        dlt = getattr(a, f) - getattr(b, f)
        s += float(np.sum(dlt * dlt))
    return rho * s


def primal_residuals(X: np.ndarray, st: State, pr: Problem) -> Tuple[float, float]:
    """||B X - P1|| and ||X - P2||: how far the iterate is from the constraints P1 = B X and
    P2 = X of the split problem eq. (fusionoptim), after the step that produced X and st."""
    r2 = X - st.P2
    if pr.fused:                       # no P1 = B X constraint in the fused-S splitting
        return 0.0, float(np.sqrt(np.sum(r2 * r2)))
    r1 = blur(X, pr.b) - st.P1
    return float(np.sqrt(np.sum(r1 * r1))), float(np.sqrt(np.sum(r2 * r2)))


@dataclasses.dataclass
class Monitor:
    """What is recorded after an iteration: the objective of eq. (mainoptim) and its terms at
    X^{(t)} (the quantity plotted against t in Fig. "objective_conv"), and the primal
    residuals of the constraints of eq. (fusionoptim)."""
    iteration: int
    objective: float
    data_l: float
    data_h: float
    reg: float
    r1: float
    r2: float


def monitor(t: int, X: np.ndarray, st: State, Yl: np.ndarray, Yh: np.ndarray, pr: Problem,
            omega: Optional[np.ndarray] = None) -> Monitor:
    a, b, c = objective_terms(X, Yl, Yh, pr, omega)
    r1, r2 = primal_residuals(X, st, pr)
    return Monitor(iteration=t, objective=a + b + c, data_l=a, data_h=b, reg=c, r1=r1, r2=r2)


@dataclasses.dataclass
class Result:
    X: np.ndarray            # the iterate X^{(T)} (L_s bands)
    state: State
    objective: List[float]
    residual: List[float]
    Z: Optional[np.ndarray] = None   # Z = X E (L bands)
    monitor: Optional[List[Monitor]] = None


def solve(Yl: np.ndarray, Yh: np.ndarray, pr: Problem, iters: int, init: str = "upsample",
          track: bool = False, state: Optional[Tuple[np.ndarray, State]] = None,
          monitor_every: int = 0, workers: int = 1) -> Result:
    """Run ``iters`` ADMM iterations; X^{(iters)} and Z = X E.  With monitor_every = N > 0,
    ``monitor`` holds a record after iterations N, 2N, ... and after the last one.
    ``workers`` > 1 runs the (tau, k) loops of the paper's splitting on that many threads,
    with results bit-identical to one worker."""
    if workers > 1 and not pr.fused:
        with ThreadPoolExecutor(max_workers=workers) as pool:
            return _solve(Yl, Yh, pr, iters, init, track, state, monitor_every, pool)
    return _solve(Yl, Yh, pr, iters, init, track, state, monitor_every, None)


def _solve(Yl, Yh, pr, iters, init, track, state, monitor_every, pool) -> Result:
    Yl = Yl.astype(np.float64)
    Yh = Yh.astype(np.float64)
    den = denominator(pr.p, pr.q, pr.b, pr.window, pr.K)
    omega = weights(Yh, pr.window, pr.K, pr.h, pr.unweighted)
    mu = pr.lam * omega / pr.rho
    F = p2_matrix(pr)
    X, st = state if state is not None else initial_state(Yl, pr, init)
    if pr.fused:
        assert pr.E is None, "the fused-S variant is built for E = I"
        a = fused_denominator(pr.p, pr.q, pr.window, pr.K)
        C0 = blur_T(decimate_T(Yl, pr.d, pr.p, pr.q), pr.b) / pr.rho
        step = lambda st_: admm_step_fused(st_, Yl, Yh, pr, a, C0, mu, F)
    else:
        step = lambda st_: admm_step(st_, Yl, Yh, pr, den, mu, F, pool)
    objs: List[float] = []
    res: List[float] = []
    mons: List[Monitor] = []
    for t in range(1, iters + 1):
        X, nst = step(st)
        if track:
            objs.append(objective(X, Yl, Yh, pr, omega))
            res.append(fixed_point_residual(nst, st, pr.rho))
        if monitor_every > 0 and (t % monitor_every == 0 or t == iters):
            mons.append(monitor(t, X, nst, Yl, Yh, pr, omega))
        st = nst
    return Result(X=X, state=st, objective=objs, residual=res, Z=compose(X, pr),
                  monitor=mons if monitor_every > 0 else None)


# --------------------------------------------------- first two iterations, few bands
def two_iterations_bands(Yl: np.ndarray, Yh: np.ndarray, pr: Problem,
                         bands: Sequence[int]) -> np.ndarray:
    """X^{(2)} restricted to ``bands``, from the default initial values, for images too
    large to hold Q and Sigma for every band.

    It is the same arithmetic as two calls of ``admm_step``: with Q^{(0)} = Sigma^{(0)} = 0
    the first X-update needs no regulariser term, and X^{(2)}_c needs the regulariser
    term of C^{(1)} only for band c.  The bands are coupled by the P2-update alone,
    which is computed for all bands.  Without a subspace basis only."""
    assert pr.E is None
    Yl = Yl.astype(np.float64)
    Yh = Yh.astype(np.float64)
    den = denominator(pr.p, pr.q, pr.b, pr.window, pr.K)
    omega = weights(Yh, pr.window, pr.K, pr.h, pr.unweighted)
    mu = pr.lam * omega / pr.rho
    F = p2_matrix(pr)
    X0 = upsample_nn(Yl, pr.d)
    P1, P2 = blur(X0, pr.b), X0
    zero = np.zeros_like(X0)
    # iteration 1: C^{(0)} = B^T(P1 + 0) + P2 + 0 + sum D^T(0 + 0)
    X1 = x_update(blur_T(P1, pr.b) + P2, den)
    BX1 = blur(X1, pr.b)
    P1 = p1_update(BX1, zero, Yl, pr)
    P2 = p2_update(X1, zero, Yh, pr, F)
    Lam1 = zero - (BX1 - P1)
    Lam2 = zero - (X1 - P2)
    bands = list(bands)
    X1b = X1[bands]
    C = (blur_T(P1 + Lam1, pr.b) + P2 + Lam2)[bands]
    for n, t in enumerate(pr.window):
        for k in pr.patch:
            DX = D(X1b, t, k)
            Qn = soft_threshold(DX - 0.0, mu[n][None])
            Sn = 0.0 - (DX - Qn)
            C += D_T(Qn + Sn, t, k)
    return x_update(C, den)
