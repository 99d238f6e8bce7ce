"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here retypes an oracle formula.  Each test checks the oracle against something
independent of it: brute force from the definitions on tiny inputs (explicit index
arithmetic and pure-Python loops), closed forms, dense linear algebra, optimality
conditions of each subproblem, the ADMM invariants of the Appendix, and the optimum
reached by an independent primal-dual solver.  Shapes are non-square, the blur is not
symmetric and R is not symmetric, so that a transposed operand or a swapped index shows.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import nlpr_oracle as o

RNG = np.random.default_rng(12345)


# ------------------------------------------------ independent dense operators (tests only)
def idx(i1, i2, q):
    return i1 * q + i2


def dense_shift_diff(p, q, tau, k):
    """Matrix of D_{tau k} on one band: row i has +1 at i-k and -1 at i-tau-k (mod p, q)."""
    n = p * q
    M = np.zeros((n, n))
    for i1 in range(p):
        for i2 in range(q):
            r = idx(i1, i2, q)
            M[r, idx((i1 - k[0]) % p, (i2 - k[1]) % q, q)] += 1.0
            M[r, idx((i1 - tau[0] - k[0]) % p, (i2 - tau[1] - k[1]) % q, q)] -= 1.0
    return M


def dense_blur(p, q, b):
    """Matrix of the circular convolution (b * x)(i) = sum_m b(m) x(i - m) on one band."""
    r1, r2 = b.shape[0] // 2, b.shape[1] // 2
    n = p * q
    M = np.zeros((n, n))
    for i1 in range(p):
        for i2 in range(q):
            for a in range(-r1, r1 + 1):
                for c in range(-r2, r2 + 1):
                    M[idx(i1, i2, q), idx((i1 - a) % p, (i2 - c) % q, q)] += b[a + r1, c + r2]
    return M


def dense_decimate(p, q, d):
    rows = [(a, c) for a in range(0, p, d) for c in range(0, q, d)]
    M = np.zeros((len(rows), p * q))
    for r, (a, c) in enumerate(rows):
        M[r, idx(a, c, q)] = 1.0
    return M


def vec(X):
    """Planar [L][p][q] -> the paper's n x L matrix, flattened column-major by band."""
    return X.reshape(X.shape[0], -1).T


def rand_blur(r, rng=None):
    b = (RNG if rng is None else rng).uniform(0.1, 1.0, size=(2 * r + 1, 2 * r + 1))
    return b / b.sum()          # deliberately not symmetric


def tiny_problem(p=6, q=8, L=3, Lh=2, d=2, r=1, K=1, S=1, lam=0.05, rho=0.7, lam1=0.8,
                 h=0.9, unweighted=False, local=False, seed=0, Ls=None):
    rng = np.random.default_rng(seed)
    E = None if Ls is None else rng.standard_normal((Ls, L))    # general (not orthonormal) basis
    pr = o.Problem(p=p, q=q, L=L, d=d, b=rand_blur(r, rng), R=rng.uniform(0.05, 1.0, size=(L, Lh)),
                   K=K, S=S, lam=lam, rho=rho, h=h, lam1=lam1, unweighted=unweighted,
                   local=local, E=E)
    Yl = rng.uniform(0, 1, size=(L, p // d, q // d))
    Yh = rng.uniform(0, 1, size=(Lh, p, q))
    return pr, Yl, Yh


# ------------------------------------------------------------- definitions, brute force
def test_shift_and_difference_operator_brute_force():
    p, q, L = 5, 7, 2
    X = RNG.standard_normal((L, p, q))
    for tau, k in [((1, 2), (0, 0)), ((-2, 1), (1, -1)), ((0, -3), (2, 2))]:
        got = o.D(X, tau, k)
        for c, i1, i2 in itertools.product(range(L), range(p), range(q)):
            want = X[c, (i1 - k[0]) % p, (i2 - k[1]) % q] - \
                X[c, (i1 - tau[0] - k[0]) % p, (i2 - tau[1] - k[1]) % q]
            assert got[c, i1, i2] == pytest.approx(want, abs=1e-14)


def test_blur_brute_force_and_adjoint():
    p, q = 6, 9
    b = rand_blur(2)
    X = RNG.standard_normal((2, p, q))
    Mb = dense_blur(p, q, b)
    for c in range(2):
        np.testing.assert_allclose(o.blur(X, b)[c].ravel(), Mb @ X[c].ravel(), atol=1e-13)
        np.testing.assert_allclose(o.blur_T(X, b)[c].ravel(), Mb.T @ X[c].ravel(), atol=1e-13)


def test_adjointness_of_every_operator():
    p, q, L, Lh, d = 6, 8, 3, 2, 2
    b = rand_blur(1)
    R = RNG.standard_normal((L, Lh))
    x = RNG.standard_normal((L, p, q))
    y = RNG.standard_normal((L, p, q))
    ip = lambda a, c: float(np.sum(a * c))
    assert ip(o.blur(x, b), y) == pytest.approx(ip(x, o.blur_T(y, b)), rel=1e-12)
    for tau, k in [((1, -1), (0, 1)), ((2, 0), (-1, -1)), ((0, 1), (1, 0))]:
        assert ip(o.D(x, tau, k), y) == pytest.approx(ip(x, o.D_T(y, tau, k)), rel=1e-12)
    yl = RNG.standard_normal((L, p // d, q // d))
    assert ip(o.decimate(x, d), yl) == pytest.approx(ip(x, o.decimate_T(yl, d, p, q)), rel=1e-12)
    yh = RNG.standard_normal((Lh, p, q))
    # <X R, Yh> = <X, Yh R^T> with the paper's n x L matrices
    lhs = ip(o.spectral(x, R), yh)
    rhs = float(np.sum(vec(x) * (vec(yh) @ R.T)))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_sampling_mask_identities():
    # eq. (maskprop): S^T S S^T = S^T and (S^T S)^2 = S^T S
    p, q, d = 8, 12, 4
    S = dense_decimate(p, q, d)
    StS = S.T @ S
    np.testing.assert_array_equal(StS @ S.T, S.T)
    np.testing.assert_array_equal(StS @ StS, StS)
    np.testing.assert_array_equal(np.diag(StS).reshape(p, q), o.sampling_mask(p, q, d))


def patch_vector(Y, i, K):
    """P_i(Y): X_c(i - k) for (k, c) in Lambda, in one fixed ordering (Sec. Definition)."""
    Lh, p, q = Y.shape
    return np.array([Y[c, (i[0] - a) % p, (i[1] - b) % q]
                     for a in range(-K, K + 1) for b in range(-K, K + 1) for c in range(Lh)])


def test_weights_brute_force_from_patch_vectors():
    p, q, Lh, K, S, h = 6, 7, 2, 1, 2, 0.8
    Y = RNG.uniform(0, 1, size=(Lh, p, q))
    W = o.search_window(S)
    om = o.weights(Y, W, K, h)
    for n, t in enumerate(W):
        for i1, i2 in itertools.product(range(p), range(q)):
            diff = patch_vector(Y, (i1, i2), K) - patch_vector(Y, ((i1 - t[0]) % p, (i2 - t[1]) % q), K)
            want = math.exp(-float(diff @ diff) / (h * h))
            assert om[n, i1, i2] == pytest.approx(want, rel=1e-12, abs=1e-300)


def test_weights_invariants():
    p, q, Lh, K, S = 7, 6, 3, 2, 2
    Y = RNG.uniform(0, 1, size=(Lh, p, q))
    W = o.search_window(S)
    om = o.weights(Y, W, K, 2.0)
    n0 = W.index((0, 0))
    np.testing.assert_array_equal(om[n0], 1.0)                         # omega_{i,0} = 1
    for n, t in enumerate(W):                                          # omega_{i-tau,-tau} = omega_{i tau}
        m = W.index((-t[0], -t[1]))
        np.testing.assert_allclose(o.shift(om[m], t), om[n], rtol=1e-13)
    const = np.full((Lh, p, q), 0.37)
    np.testing.assert_array_equal(o.weights(const, W, K, 0.5), 1.0)  # constant guide -> 1
    assert np.all(om <= 1.0) and np.all(om > 0.0)


def test_regulariser_patch_form_equals_filter_form():
    # eq. (reg1) with explicit patch vectors == eq. (regfilt1)
    p, q, L, Lh, K, S = 5, 6, 2, 1, 1, 1
    X = RNG.standard_normal((L, p, q))
    Y = RNG.uniform(0, 1, size=(Lh, p, q))
    W = o.search_window(S)
    om = o.weights(Y, W, K, 0.6)
    want = 0.0
    for n, t in enumerate(W):
        for i1, i2 in itertools.product(range(p), range(q)):
            dv = patch_vector(X, (i1, i2), K) - patch_vector(X, ((i1 - t[0]) % p, (i2 - t[1]) % q), K)
            want += om[n, i1, i2] * float(np.sum(np.abs(dv)))
    assert o.regulariser(X, om, W, K) == pytest.approx(want, rel=1e-12)


def test_unweighted_patch_regulariser_is_P_times_pixel_regulariser():
    # omega = 1: the patch sum re-indexes the pixel sum on the periodic domain (ablation C2 vs C4)
    p, q, L = 6, 7, 2
    X = RNG.standard_normal((L, p, q))
    for K, S in [(1, 1), (2, 2)]:
        W = o.search_window(S)
        ones = np.ones((len(W), p, q))
        patch = o.regulariser(X, ones, W, K)
        pixel = o.regulariser(X, ones, W, 0)
        assert patch == pytest.approx((2 * K + 1) ** 2 * pixel, rel=1e-12)


# ------------------------------------------------------------------ X-update / Fourier
def test_denominator_closed_form():
    # |d^_{tau 0}(w)|^2 = 2 - 2 cos(2 pi (w1 tau1 / p + w2 tau2 / q)); |b^|^2 by a direct DFT sum
    p, q, K, S = 8, 6, 1, 2
    b = rand_blur(1)
    W = o.search_window(S)
    w1 = np.arange(p)[:, None]
    w2 = np.arange(q)[None, :]
    bh = np.zeros((p, q), dtype=complex)
    r = 1
    for a in range(-r, r + 1):
        for c in range(-r, r + 1):
            bh += b[a + r, c + r] * np.exp(-2j * np.pi * (w1 * a / p + w2 * c / q))
    # sum over the square window factorises into Dirichlet kernels:
    # sum_{tau in [-S,S]^2} cos(A t1 + B t2) = D_S(A) D_S(B), D_S(x) = sum_{t=-S}^{S} cos(t x)
    A = 2 * np.pi * w1 / p
    B = 2 * np.pi * w2 / q
    DS = lambda x: sum(np.cos(t * x) for t in range(-S, S + 1))
    sum_d = 2 * len(W) - 2 * DS(A) * DS(B)
    want = 1 + np.abs(bh) ** 2 + (2 * K + 1) ** 2 * sum_d
    np.testing.assert_allclose(o.denominator(p, q, b, W, K), want, rtol=1e-12)


def test_shift_property_of_difference_filters():
    # |d^_{tau k}| = |d^_{tau 0}| (Sec. "Patch variation using convolutions")
    p, q = 6, 10
    for tau, k in [((1, 2), (1, -1)), ((-2, 3), (2, 0))]:
        def dft_of(t, kk):
            g = np.zeros((p, q))
            g[kk[0] % p, kk[1] % q] += 1
            g[(t[0] + kk[0]) % p, (t[1] + kk[1]) % q] -= 1
            return np.abs(np.fft.fft2(g))
        np.testing.assert_allclose(dft_of(tau, k), dft_of(tau, (0, 0)), atol=1e-12)


@pytest.mark.parametrize("p,q,K,S", [(6, 8, 1, 1), (8, 6, 0, 2), (5, 7, 1, 2)])
def test_x_update_equals_dense_solve(p, q, K, S):
    # eq. (x_linear_system_main) solved densely vs the Fourier solve of eq. (inv)
    b = rand_blur(1)
    W = o.search_window(S)
    P = o.patch_offsets(K)
    n = p * q
    Mb = dense_blur(p, q, b)
    A = np.eye(n) + Mb.T @ Mb
    for t in W:
        for k in P:
            Dm = dense_shift_diff(p, q, t, k)
            A += Dm.T @ Dm
    C = RNG.standard_normal((2, p, q))
    X = o.x_update(C, o.denominator(p, q, b, W, K))
    for c in range(2):
        np.testing.assert_allclose(X[c].ravel(), np.linalg.solve(A, C[c].ravel()), atol=1e-11)


# ----------------------------------------------------------------- proximal / subproblems
def test_soft_threshold_is_prox_of_weighted_l1():
    grid = np.linspace(-3, 3, 600001)
    for v, mu in [(1.3, 0.4), (-0.2, 0.5), (0.5, 0.5), (-2.1, 0.05), (0.7, 0.0)]:
        f = np.abs(grid) + (grid - v) ** 2 / (2 * mu) if mu > 0 else None
        want = grid[np.argmin(f)] if mu > 0 else v
        assert float(o.soft_threshold(np.array(v), mu)) == pytest.approx(want, abs=2e-5)
    # the dual after the Q-update is -clip(V, mu), and Q + Sigma = V - 2 clip(V, mu)
    V = RNG.standard_normal(1000)
    mu = RNG.uniform(0, 1, 1000)
    Q = o.soft_threshold(V, mu)
    sig = -(V - Q)   # Sigma^{t+1} = Sigma^t - (D X - Q) with V = D X - Sigma^t
    np.testing.assert_allclose(sig, -np.clip(V, -mu, mu), atol=1e-15)


@pytest.mark.parametrize("Ls", [None, 2])
def test_p1_update_solves_its_normal_equation(Ls):
    # eq. (P1grad): S^T S P1 E E^T + rho P1 = S^T Y_l E^T + rho (B X - Lambda1)
    pr, Yl, Yh = tiny_problem(Ls=Ls)
    E = np.eye(pr.L) if Ls is None else pr.E
    BX = RNG.standard_normal((pr.Ls, pr.p, pr.q))
    Lam1 = RNG.standard_normal((pr.Ls, pr.p, pr.q))
    P1 = o.p1_update(BX, Lam1, Yl, pr)
    S = dense_decimate(pr.p, pr.q, pr.d)
    lhs = (S.T @ S) @ vec(P1) @ E @ E.T + pr.rho * vec(P1)
    rhs = S.T @ vec(Yl) @ E.T + pr.rho * (vec(BX) - vec(Lam1))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


@pytest.mark.parametrize("Ls", [None, 2])
def test_p2_update_zeroes_its_gradient(Ls):
    # gradient of lambda1/2 ||Y_h - P2 E R||^2 + rho/2 ||P2 + Lambda2 - X||^2 vanishes
    pr, Yl, Yh = tiny_problem(Ls=Ls)
    ER = pr.R if Ls is None else pr.E @ pr.R
    X = RNG.standard_normal((pr.Ls, pr.p, pr.q))
    Lam2 = RNG.standard_normal((pr.Ls, pr.p, pr.q))
    P2 = vec(o.p2_update(X, Lam2, Yh, pr))
    g = -pr.lam1 * (vec(Yh) - P2 @ ER) @ ER.T + pr.rho * (P2 + vec(Lam2) - vec(X))
    np.testing.assert_allclose(g, 0.0, atol=1e-12)


def _full_step(pr, Yl, Yh, iters=3):
    den = o.denominator(pr.p, pr.q, pr.b, pr.window, pr.K)
    om = o.weights(Yh, pr.window, pr.K, pr.h, pr.unweighted)
    mu = pr.lam * om / pr.rho
    F = o.p2_matrix(pr)
    X, st = o.initial_state(Yl, pr)
    for _ in range(iters):
        X, st = o.admm_step(st, Yl, Yh, pr, den, mu, F)
    return X, st, mu, den, F


def test_subspace_admm_reaches_the_optimum_of_an_independent_solver():
    """The low-rank form Z = X E (Sec. "Variational models"): the ADMM optimum over X equals
    that of the primal-dual solver on the same dense problem."""
    pr, Yl, Yh = tiny_problem(p=4, q=6, L=3, Lh=1, d=2, K=1, S=1, lam=0.02, h=0.7, Ls=2,
                              rho=0.3)
    H, bb, c0, G, w = _dense_problem(pr, Yl, Yh)
    x_pd = _pdhg(H, bb, G, w, 10000)
    f_pd = _dense_objective(x_pd, H, bb, c0, G, w)
    res = o.solve(Yl, Yh, pr, 4000)
    f_admm = _dense_objective(vec(res.X).T.ravel(), H, bb, c0, G, w)
    assert o.objective(res.X, Yl, Yh, pr) == pytest.approx(f_admm, rel=1e-12)
    assert f_admm == pytest.approx(f_pd, rel=1e-9)
    # Z = X E
    np.testing.assert_allclose(vec(res.Z), vec(res.X) @ pr.E, atol=1e-14)


def test_initial_state_by_index_loops():
    """The start (the paper names the initial values but does not give them; the reading
    is X0 = nearest-neighbour upsample of Y_l, P1 = B X0, P2 = X0, all else 0), checked
    with pure-Python index loops and the dense blur matrix, on a non-square image with
    decimation 3 and an asymmetric blur."""
    pr, Yl, Yh = tiny_problem(p=6, q=9, L=2, d=3, r=1)
    X0, st = o.initial_state(Yl, pr)
    ref = np.zeros((pr.L, pr.p, pr.q))
    for c in range(pr.L):
        for i1 in range(pr.p):
            for i2 in range(pr.q):
                ref[c, i1, i2] = Yl[c, i1 // pr.d, i2 // pr.d]
    np.testing.assert_array_equal(X0, ref)
    Bm = dense_blur(pr.p, pr.q, pr.b)
    for c in range(pr.L):
        np.testing.assert_allclose(st.P1[c].ravel(), Bm @ ref[c].ravel(), atol=1e-14)
    np.testing.assert_array_equal(st.P2, ref)
    for f in ("Q", "Sig", "Lam1", "Lam2"):
        assert not np.any(getattr(st, f)), f
    assert st.Q.shape == st.Sig.shape == (len(pr.window), len(pr.patch), pr.L, pr.p, pr.q)
    Xz, sz = o.initial_state(Yl, pr, init="zero")
    for a in (Xz, sz.P1, sz.P2, sz.Q, sz.Sig, sz.Lam1, sz.Lam2):
        assert not np.any(a)


def test_initial_state_hand_computed():
    """A 2 x 2 Y_l with d = 2 and the two-tap blur b(0, 0) = b(0, 1) = 1/2, written out by
    hand: X0 repeats each low-resolution pixel over its 2 x 2 block, and
    P1(i) = (X0(i1, i2) + X0(i1, i2 - 1)) / 2 with the column index taken mod 4."""
    b = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5], [0.0, 0.0, 0.0]])
    pr = o.Problem(p=4, q=4, L=1, d=2, b=b, R=np.ones((1, 1)), K=0, S=1, lam=0.1,
                   rho=0.5, h=1.0)
    Yl = np.array([[[1.0, 2.0], [3.0, 4.0]]])
    X0, st = o.initial_state(Yl, pr)
    np.testing.assert_array_equal(X0[0], [[1, 1, 2, 2], [1, 1, 2, 2], [3, 3, 4, 4], [3, 3, 4, 4]])
    np.testing.assert_allclose(st.P1[0], [[1.5, 1, 1.5, 2], [1.5, 1, 1.5, 2],
                                          [3.5, 3, 3.5, 4], [3.5, 3, 3.5, 4]], atol=1e-15)
    np.testing.assert_array_equal(st.P2[0], X0[0])


def test_subspace_start_is_the_least_squares_coefficient_image():
    pr, Yl, Yh = tiny_problem(Ls=2)
    X0, _ = o.initial_state(Yl, pr)
    up = np.repeat(np.repeat(Yl, pr.d, axis=-2), pr.d, axis=-1)
    coef, *_ = np.linalg.lstsq(pr.E.T, vec(up).T, rcond=None)     # min ||X E - up||
    np.testing.assert_allclose(vec(X0), coef.T, atol=1e-12)


def test_admm_step_subproblem_optimality():
    """Each update of one ADMM step satisfies the optimality condition of its subproblem
    (eqs. (x_update_problem), (P1_update_problem), (P2_update_problem), (Qj_update_problem))
    and the dual updates, checked with independent dense operators."""
    pr, Yl, Yh = tiny_problem()
    _, st, mu, den, F = _full_step(pr, Yl, Yh, iters=2)
    X, nst = o.admm_step(st, Yl, Yh, pr, den, mu, F)
    n = pr.p * pr.q
    Mb = dense_blur(pr.p, pr.q, pr.b)
    S = dense_decimate(pr.p, pr.q, pr.d)
    W, P = pr.window, pr.patch
    # X-subproblem gradient: B^T(BX - P1 - L1) + (X - P2 - L2) + sum D^T(DX - Q - Sig) = 0
    g = Mb.T @ (Mb @ vec(X) - vec(st.P1) - vec(st.Lam1)) + (vec(X) - vec(st.P2) - vec(st.Lam2))
    for a, t in enumerate(W):
        for m, k in enumerate(P):
            Dm = dense_shift_diff(pr.p, pr.q, t, k)
            g += Dm.T @ (Dm @ vec(X) - vec(st.Q[a, m]) - vec(st.Sig[a, m]))
    np.testing.assert_allclose(g, 0.0, atol=1e-10)
    BX = Mb @ vec(X)
    # P1: S^T(S P1 - Y_l) + rho (P1 - BX + L1) = 0
    g1 = S.T @ (S @ vec(nst.P1) - vec(Yl)) + pr.rho * (vec(nst.P1) - BX + vec(st.Lam1))
    np.testing.assert_allclose(g1, 0.0, atol=1e-11)
    # P2: -lam1 (Y_h - P2 R) R^T + rho (P2 + L2 - X) = 0
    g2 = -pr.lam1 * (vec(Yh) - vec(nst.P2) @ pr.R) @ pr.R.T + pr.rho * (vec(nst.P2) + vec(st.Lam2) - vec(X))
    np.testing.assert_allclose(g2, 0.0, atol=1e-11)
    # Q: 0 in lam2 w d|Q| + rho (Q - (DX - Sig))
    for a, t in enumerate(W):
        for m, k in enumerate(P):
            Dm = dense_shift_diff(pr.p, pr.q, t, k)
            qt = Dm @ vec(X) - vec(st.Sig[a, m])
            Qv = vec(nst.Q[a, m])
            thr = np.repeat(vec(mu[a][None]), pr.L, axis=1)   # lam2 w / rho per pixel
            nz = Qv != 0
            np.testing.assert_allclose((Qv - qt)[nz], -(thr * np.sign(Qv))[nz], atol=1e-12)
            assert np.all(np.abs(qt[~nz]) <= thr[~nz] + 1e-12)
            # dual: Sig+ = Sig - (DX - Q)
            np.testing.assert_allclose(vec(nst.Sig[a, m]),
                                       vec(st.Sig[a, m]) - (Dm @ vec(X) - Qv), atol=1e-12)
    np.testing.assert_allclose(vec(nst.Lam1), vec(st.Lam1) - (BX - vec(nst.P1)), atol=1e-12)
    np.testing.assert_allclose(vec(nst.Lam2), vec(st.Lam2) - (vec(X) - vec(nst.P2)), atol=1e-12)


# ------------------------------------------------------------------- ADMM invariants
def test_fixed_point_residual_is_non_increasing():
    # ADMM: rho(||dV||^2 + ||dU||^2) is non-increasing in t (He & Yuan 2015), with the
    # V / U grouping of the Appendix.
    pr, Yl, Yh = tiny_problem(p=8, q=6, L=2, Lh=1, lam=0.2, rho=0.3, h=0.5)
    res = o.solve(Yl, Yh, pr, 60, track=True).residual
    for a, b in zip(res, res[1:]):
        assert b <= a * (1 + 1e-10) + 1e-300


def test_two_iteration_band_form_equals_full_iteration():
    pr, Yl, Yh = tiny_problem(p=8, q=12, L=4, Lh=2, K=1, S=2)
    full = o.solve(Yl, Yh, pr, 2).X
    part = o.two_iterations_bands(Yl, Yh, pr, [0, 3])
    np.testing.assert_allclose(part, full[[0, 3]], rtol=1e-12, atol=1e-13)


def _dense_problem(pr, Yl, Yh):
    """H, b, c, G, w of f(x) = 1/2 x^T H x - b^T x + c and phi = sum_j w_j |(G x)_j|, for
    x the band-major vector of X (Z = X E)."""
    n, L = pr.p * pr.q, pr.L
    E = np.eye(L) if pr.E is None else pr.E
    Ls = E.shape[0]
    Mb = dense_blur(pr.p, pr.q, pr.b)
    S = dense_decimate(pr.p, pr.q, pr.d)
    A1 = np.kron(E.T, S @ Mb)                      # S B (X E), band-major
    A2 = np.kron((E @ pr.R).T, np.eye(n))          # (X E R), band-major
    L = Ls
    y1 = vec(Yl).T.ravel()
    y2 = vec(Yh).T.ravel()
    H = A1.T @ A1 + pr.lam1 * A2.T @ A2
    bb = A1.T @ y1 + pr.lam1 * A2.T @ y2
    c0 = 0.5 * y1 @ y1 + 0.5 * pr.lam1 * y2 @ y2
    om = o.weights(Yh, pr.window, pr.K, pr.h, pr.unweighted)
    Gs, ws = [], []
    for a, t in enumerate(pr.window):
        for k in pr.patch:
            Gs.append(np.kron(np.eye(L), dense_shift_diff(pr.p, pr.q, t, k)))
            ws.append(np.tile(om[a].ravel(), L) * pr.lam)
    return H, bb, c0, np.vstack(Gs), np.concatenate(ws)


def _dense_objective(x, H, bb, c0, G, w):
    return 0.5 * x @ H @ x - bb @ x + c0 + float(np.sum(w * np.abs(G @ x)))


def _pdhg(H, bb, G, w, iters):
    """Chambolle-Pock primal-dual hybrid gradient (Chambolle & Pock 2011, Algorithm 1,
    theta = 1) for min_x 1/2 x^T H x - b^T x + sum_j w_j |(G x)_j|."""
    n = H.shape[0]
    Lg = np.linalg.norm(G, 2)
    tau = sig = 0.99 / Lg
    solve = np.linalg.inv(np.eye(n) + tau * H)
    x = np.zeros(n)
    xb = x.copy()
    y = np.zeros(G.shape[0])
    for _ in range(iters):
        y = np.clip(y + sig * (G @ xb), -w, w)
        xn = solve @ (x - tau * (G.T @ y) + tau * bb)
        xb = 2 * xn - x
        x = xn
    return x


def test_admm_reaches_the_optimum_of_an_independent_solver():
    """Theorem 1: from any initialisation and any rho the iterates reach a minimiser of
    eq. (ouroptim).  Compare optimal values with a primal-dual solver on dense matrices."""
    pr, Yl, Yh = tiny_problem(p=4, q=6, L=2, Lh=1, d=2, K=1, S=1, lam=0.02, h=0.7)
    H, bb, c0, G, w = _dense_problem(pr, Yl, Yh)
    x_pd = _pdhg(H, bb, G, w, 10000)
    f_pd = _dense_objective(x_pd, H, bb, c0, G, w)
    for rho, iters in ((0.3, 4000), (1.0, 8000)):
        pr.rho = rho
        X = o.solve(Yl, Yh, pr, iters).X
        f_admm = _dense_objective(vec(X).T.ravel(), H, bb, c0, G, w)
        # the dense objective and the oracle's own objective agree
        assert o.objective(X, Yl, Yh, pr) == pytest.approx(f_admm, rel=1e-12)
        assert f_admm == pytest.approx(f_pd, rel=1e-10)


def _brute_force_fused_minimiser(y, edges, w):
    """Exact minimiser of 1/2 ||y - x||^2 + sum_e w_e |x_a - x_b| by enumerating the branch of
    every pair: x_a > x_b, x_a < x_b or x_a = x_b.  A pattern holds at the optimum when its
    optimality system is feasible (stationarity, with subgradients z_e in [-w_e, w_e] on the
    fused pairs and the given signs on the others), which is a linear program.  The objective
    is strictly convex, so every feasible pattern gives the same x."""
    from scipy.optimize import linprog
    n, sols = len(y), []
    for pat in itertools.product((1, -1, 0), repeat=len(edges)):
        fused = [k for k, sg in enumerate(pat) if sg == 0]
        nf = len(fused)
        A_eq = np.zeros((n + nf, n + nf))
        b_eq = np.concatenate([np.asarray(y, dtype=float), np.zeros(nf)])
        A_eq[:n, :n] = np.eye(n)
        A_ub, b_ub = [], []
        for k, (a, b) in enumerate(edges):
            if pat[k]:
                b_eq[a] -= w[k] * pat[k]
                b_eq[b] += w[k] * pat[k]
                row = np.zeros(n + nf)
                row[a], row[b] = -pat[k], pat[k]          # pat (x_a - x_b) >= 0
                A_ub.append(row)
                b_ub.append(0.0)
        for j, k in enumerate(fused):
            a, b = edges[k]
            A_eq[a, n + j] += 1.0
            A_eq[b, n + j] -= 1.0
            A_eq[n + j, a], A_eq[n + j, b] = 1.0, -1.0    # x_a = x_b
        res = linprog(np.zeros(n + nf), A_ub=np.array(A_ub) if A_ub else None,
                      b_ub=np.array(b_ub) if b_ub else None, A_eq=A_eq, b_eq=b_eq,
                      bounds=[(None, None)] * n + [(-w[k], w[k]) for k in fused], method="highs")
        if res.status == 0:
            sols.append(res.x[:n])
    assert sols
    X = np.array(sols)
    assert np.ptp(X, axis=0).max() <= 1e-9        # one minimiser
    return X[0]


@pytest.mark.parametrize("p,q,lam", [(1, 4, 0.02), (1, 4, 0.05), (2, 2, 0.02), (1, 6, 0.05)])
def test_admm_reaches_the_brute_force_active_set_solution(p, q, lam):
    """With d = 1, B = I and lambda_1 = 0, eq. (ouroptim) is the weighted nonlocal TV
    denoising of Y_l: 1/2 ||Y_l - X||^2 + lambda_2 sum_{tau in W} sum_i omega_{i tau}
    |X(i) - X(i - tau)| (patch 1 x 1).  Its exact minimiser comes from enumerating the branch of
    every pixel pair; the cases cover no fusion (1 x 4, lambda_2 = 0.02) and partial fusion
    (3 distinct values of 4 or 6).  Theorem 1: ADMM reaches it from any start and rho."""
    rng = np.random.default_rng(7)
    pr = o.Problem(p=p, q=q, L=1, d=1, b=np.ones((1, 1)), R=np.ones((1, 1)), K=0, S=1, lam=lam,
                   rho=1.0, h=0.8, lam1=0.0)
    Yl = rng.uniform(0, 1, (1, p, q))
    Yh = rng.uniform(0, 1, (1, p, q))
    om = o.weights(Yh, pr.window, pr.K, pr.h, pr.unweighted)
    pix = lambda a, b: (a % p) * q + (b % q)
    wsum = {}
    for n, t in enumerate(pr.window):
        for i1 in range(p):
            for i2 in range(q):
                u, v = pix(i1, i2), pix(i1 - t[0], i2 - t[1])
                if u != v:
                    key = (min(u, v), max(u, v))
                    wsum[key] = wsum.get(key, 0.0) + lam * om[n][i1, i2]
    edges = sorted(wsum)
    xs = _brute_force_fused_minimiser(Yl.ravel(), edges, np.array([wsum[e] for e in edges]))
    for rho, iters in ((1.0, 3000), (0.3, 6000)):
        pr.rho = rho
        X = o.solve(Yl, Yh, pr, iters, init="zero").X.ravel()
        assert np.abs(X - xs).max() <= 1e-9


@pytest.mark.parametrize("S,rho,iters", [(0, 0.5, 500), (1, 0.1, 3000)])
def test_lambda2_zero_with_square_R_gives_the_least_squares_solution(S, rho, iters):
    # lambda2 = 0 and an invertible L x L response: the unique minimiser solves the normal
    # equations of the two data terms of eq. (mainoptim)
    pr, Yl, Yh = tiny_problem(p=4, q=6, L=2, Lh=2, d=2, lam=0.0, rho=rho, S=S)
    H, bb, *_ = _dense_problem(pr, Yl, Yh)
    x_ls = np.linalg.solve(H, bb)
    X = o.solve(Yl, Yh, pr, iters, init="zero").X
    np.testing.assert_allclose(vec(X).T.ravel(), x_ls, atol=1e-8)


def test_objective_stabilises():
    # the objective settles within a few hundred iterations (convergence figure of the
    # experiments); ADMM does not promise a monotone objective, so only check that the
    # late changes are small next to the total decrease
    pr, Yl, Yh = tiny_problem(p=8, q=8, L=2, Lh=1, lam=0.05, rho=0.5, h=0.5)
    obj = o.solve(Yl, Yh, pr, 300, track=True).objective
    drop = obj[0] - obj[-1]
    assert drop > 0
    assert np.ptp(obj[200:]) <= 0.05 * drop


# ------------------------------------------------------------------ monitor quantities
@pytest.mark.parametrize("Ls", [None, 2])
def test_objective_terms_equal_dense_operator_forms(Ls):
    """Each term of eq. (mainoptim), from explicit matrices of S, B, R, E and D_{tau k}
    (the three terms separately, so a term moved or dropped shows)."""
    pr, Yl, Yh = tiny_problem(p=6, q=4, L=3, Lh=2, d=2, K=1, S=1, lam=0.07, lam1=0.6, Ls=Ls)
    rng = np.random.default_rng(7)
    X = rng.standard_normal((pr.Ls, pr.p, pr.q))
    n = pr.p * pr.q
    E = np.eye(pr.L) if Ls is None else pr.E
    A1 = np.kron(E.T, dense_decimate(pr.p, pr.q, pr.d) @ dense_blur(pr.p, pr.q, pr.b))
    A2 = np.kron((E @ pr.R).T, np.eye(n))
    x = vec(X).T.ravel()
    y1 = vec(Yl).T.ravel()
    y2 = vec(Yh).T.ravel()
    *_, G, w = _dense_problem(pr, Yl, Yh)
    want = (0.5 * np.sum((y1 - A1 @ x) ** 2), 0.5 * pr.lam1 * np.sum((y2 - A2 @ x) ** 2),
            float(np.sum(w * np.abs(G @ x))))
    got = o.objective_terms(X, Yl, Yh, pr)
    for g, v in zip(got, want):
        assert g == pytest.approx(v, rel=1e-12)


@pytest.mark.parametrize("Ls", [None, 2])
def test_primal_residuals_are_the_lambda_steps(Ls):
    """eqs. (dualvar1_main), (dualvar2_main): the step of Lambda1 is B X - P1 and that of
    Lambda2 is X - P2, so the residual norms equal the norms of the dual steps; B X is
    also formed with the explicit blur matrix."""
    pr, Yl, Yh = tiny_problem(p=6, q=8, L=3, Lh=2, Ls=Ls, seed=3)
    X0, st = o.initial_state(Yl, pr)
    den = o.denominator(pr.p, pr.q, pr.b, pr.window, pr.K)
    om = o.weights(Yh, pr.window, pr.K, pr.h)
    mu = pr.lam * om / pr.rho
    F = o.p2_matrix(pr)
    for _ in range(2):
        X, nst = o.admm_step(st, Yl, Yh, pr, den, mu, F)
        r1, r2 = o.primal_residuals(X, nst, pr)
        assert r1 == pytest.approx(np.linalg.norm(nst.Lam1 - st.Lam1), rel=1e-12)
        assert r2 == pytest.approx(np.linalg.norm(nst.Lam2 - st.Lam2), rel=1e-12)
        Mb = dense_blur(pr.p, pr.q, pr.b)
        BX = (Mb @ vec(X)).T.reshape(X.shape)
        assert r1 == pytest.approx(np.linalg.norm(BX - nst.P1), rel=1e-12)
        st = nst


def test_monitor_points_and_their_values():
    # records after iterations N, 2N, ... and the last; each equals the per-iteration
    # objective of the tracked run and the residuals of that iteration's state
    pr, Yl, Yh = tiny_problem(p=6, q=8, L=2, Lh=1, seed=5)
    res = o.solve(Yl, Yh, pr, 7, track=True, monitor_every=3)
    assert [m.iteration for m in res.monitor] == [3, 6, 7]
    for m in res.monitor:
        assert m.objective == pytest.approx(res.objective[m.iteration - 1], rel=1e-14)
        assert m.objective == pytest.approx(m.data_l + m.data_h + m.reg, rel=1e-14)
    last = res.monitor[-1]
    assert (last.r1, last.r2) == pytest.approx(o.primal_residuals(res.X, res.state, pr),
                                               rel=1e-14)
    assert o.solve(Yl, Yh, pr, 7).monitor is None


def test_primal_residuals_vanish_at_the_optimum():
    # Theorem 1: the constraint violations of eq. (fusionoptim) go to zero
    pr, Yl, Yh = tiny_problem(p=4, q=6, L=2, Lh=1, d=2, K=1, S=1, lam=0.02, h=0.7, rho=0.3)
    early = o.solve(Yl, Yh, pr, 20, monitor_every=20).monitor[-1]
    late = o.solve(Yl, Yh, pr, 3000, monitor_every=3000).monitor[-1]
    assert late.r1 < 1e-9 and late.r2 < 1e-9
    assert early.r1 > 1e3 * late.r1 and early.r2 > 1e3 * late.r2


# -------------------------------------------------------- fused-S X-update (S in the system)
@pytest.mark.parametrize("p,q,d,K,S", [(8, 12, 2, 1, 1), (8, 8, 4, 0, 1), (12, 8, 4, 1, 2)])
def test_fused_x_update_equals_dense_solve(p, q, d, K, S):
    """(I + sum_{tau, k} D^T D + B^T S^T S B / rho) X = C from explicit matrices."""
    pr, _, _ = tiny_problem(p=p, q=q, L=2, Lh=1, d=d, r=1, K=K, S=S, rho=0.37)
    pr.fused = True
    n = p * q
    Mb = dense_blur(p, q, pr.b)
    Sd = dense_decimate(p, q, d)
    A = np.eye(n) + Mb.T @ Sd.T @ Sd @ Mb / pr.rho
    for t in pr.window:
        for k in pr.patch:
            Dm = dense_shift_diff(p, q, t, k)
            A += Dm.T @ Dm
    C = RNG.standard_normal((2, p, q))
    want = np.stack([np.linalg.solve(A, C[c].ravel()).reshape(p, q) for c in range(2)])
    a = o.fused_denominator(p, q, pr.window, pr.K)
    np.testing.assert_allclose(o.x_update_fused(C, pr, a), want, atol=1e-11)


def test_fused_x_update_without_decimation_is_a_fourier_division():
    # d = 1: S = I, the system is diagonal in Fourier with 1 + |b^|^2 / rho + |P| sum |d^|^2
    pr, _, _ = tiny_problem(p=6, q=10, L=2, d=1, rho=0.6)
    C = RNG.standard_normal((2, 6, 10))
    bh = np.fft.fft2(o.blur_filter_grid(pr.b, 6, 10))
    a = o.fused_denominator(6, 10, pr.window, pr.K)
    den = a + np.abs(bh) ** 2 / pr.rho
    want = np.fft.ifft2(np.fft.fft2(C) / den).real
    np.testing.assert_allclose(o.x_update_fused(C, pr, a), want, atol=1e-12)


def test_fused_admm_reaches_the_optimum_of_an_independent_solver():
    """Same minimiser as the paper's splitting (Theorem 1 holds for this splitting too):
    compare the optimal value with the primal-dual solver on dense matrices."""
    pr, Yl, Yh = tiny_problem(p=4, q=6, L=2, Lh=1, d=2, K=1, S=1, lam=0.02, h=0.7)
    H, bb, c0, G, w = _dense_problem(pr, Yl, Yh)
    f_pd = _dense_objective(_pdhg(H, bb, G, w, 10000), H, bb, c0, G, w)
    pr.fused = True
    pr.rho = 0.3
    res = o.solve(Yl, Yh, pr, 4000, monitor_every=4000)
    f = _dense_objective(vec(res.X).T.ravel(), H, bb, c0, G, w)
    assert f == pytest.approx(f_pd, rel=1e-10)
    assert res.monitor[-1].r1 == 0.0 and res.monitor[-1].r2 < 1e-9


def test_thread_pool_gives_bit_identical_iterates():
    """``workers`` > 1 runs the (tau, k) loops on threads and must not change a bit: the
    terms of C are still added in the serial order."""
    pr, Yl, Yh = tiny_problem(p=8, q=12, L=3, Lh=2, d=2, K=1, S=2, lam=0.05, rho=0.3)
    a = o.solve(Yl, Yh, pr, 6, workers=1)
    b = o.solve(Yl, Yh, pr, 6, workers=5)
    np.testing.assert_array_equal(a.X, b.X)
    for f in ("P1", "P2", "Q", "Lam1", "Lam2", "Sig"):
        np.testing.assert_array_equal(getattr(a.state, f), getattr(b.state, f))
