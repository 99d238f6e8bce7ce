"""Planted mistakes in the oracle must each fail at least one pin.

Every mutation below is a plausible slip (a dropped term, a wrong sign, a swapped index or
a transposed operand).  It is patched into the oracle module on the CPU, the fast pins of
``test_oracle_pins`` are run against the mutated oracle, and at least one must fail.
"""
import numpy as np
import pytest

import test_oracle_pins as pins
from oracle import nlpr_oracle as o

FAST_PINS = [
    pins.test_shift_and_difference_operator_brute_force,
    pins.test_blur_brute_force_and_adjoint,
    pins.test_adjointness_of_every_operator,
    pins.test_weights_brute_force_from_patch_vectors,
    pins.test_weights_invariants,
    pins.test_regulariser_patch_form_equals_filter_form,
    pins.test_denominator_closed_form,
    pins.test_soft_threshold_is_prox_of_weighted_l1,
    pins.test_p1_update_solves_its_normal_equation,
    pins.test_p2_update_zeroes_its_gradient,
    pins.test_admm_step_subproblem_optimality,
    pins.test_two_iteration_band_form_equals_full_iteration,
    lambda: pins.test_x_update_equals_dense_solve(6, 8, 1, 1),
    lambda: pins.test_lambda2_zero_with_square_R_gives_the_least_squares_solution(0, 0.5, 500),
    lambda: pins.test_objective_terms_equal_dense_operator_forms(None),
    lambda: pins.test_primal_residuals_are_the_lambda_steps(None),
    lambda: pins.test_fused_x_update_equals_dense_solve(8, 12, 2, 1, 1),
    pins.test_initial_state_by_index_loops,
    pins.test_initial_state_hand_computed,
]

_orig = {name: getattr(o, name) for name in dir(o) if callable(getattr(o, name))}


def _mut_D(X, tau, k):               # wrong sign of tau
    return o.shift(X, k) - o.shift(X, (k[0] - tau[0], k[1] - tau[1]))


def _mut_DT(Y, tau, k):              # adjoint shifts the wrong way
    return o.shift(Y, k) - o.shift(Y, (tau[0] + k[0], tau[1] + k[1]))


def _mut_blurT(Y, b):                # B^T taken as B
    return _orig["blur"](Y, b)


def _mut_den(p, q, b, window, K):    # dropped |P| factor
    return _orig["denominator"](p, q, b, window, 0) if K else _orig["denominator"](p, q, b, window, 1)


def _mut_p2_matrix(pr):              # lambda1 / rho inverted
    return np.linalg.inv(np.eye(pr.L) + (pr.rho / pr.lam1) * (pr.R @ pr.R.T))


def _mut_p1(BX, Lam1, Yl, pr):       # (1 + rho) replaced by rho on the sampled pixels
    M = o.sampling_mask(pr.p, pr.q, pr.d)[None]
    StYl = o.decimate_T(Yl, pr.d, pr.p, pr.q)
    return M * (pr.rho * BX + StYl - pr.rho * Lam1) / pr.rho + (1 - M) * (BX - Lam1)


def _mut_soft(x, mu):                # half threshold
    return np.sign(x) * np.maximum(np.abs(x) - 0.5 * mu, 0.0)


def _mut_weights(Yh, window, K, h, unweighted=False):   # h instead of h^2
    if unweighted:
        return np.ones((len(window),) + Yh.shape[-2:])
    return np.stack([np.exp(-o.patch_distance(Yh, t, K) / h) for t in window])


def _mut_shift(X, t):                # shift in the wrong direction
    return np.roll(X, shift=(-t[0], -t[1]), axis=(-2, -1))


def _mut_rhs(st, pr, pool=None):     # dropped Lambda2 from the right-hand side
    C = o.blur_T(st.P1 + st.Lam1, pr.b) + st.P2
    for n, t in enumerate(pr.window):
        for m, k in enumerate(pr.patch):
            C += o.D_T(st.Q[n, m] + st.Sig[n, m], t, k)
    return C


def _mut_spectral(X, R):             # bands of R taken in reverse order
    p, q = X.shape[-2:]
    return o.from_mat(o.to_mat(X) @ R[::-1], p, q)


MUTATIONS = {
    "D": _mut_D, "D_T": _mut_DT, "blur_T": _mut_blurT, "denominator": _mut_den,
    "p2_matrix": _mut_p2_matrix, "p1_update": _mut_p1, "soft_threshold": _mut_soft,
    "weights": _mut_weights, "shift": _mut_shift, "rhs": _mut_rhs, "spectral": _mut_spectral,
}


def _admm_dual_sign(st, Yl, Yh, pr, den, mu, F, pool=None):   # dual update with the wrong sign
    X, nst = _orig["admm_step"](st, Yl, Yh, pr, den, mu, F, pool)
    BX = o.blur(X, pr.b)
    nst.Lam1 = st.Lam1 + (BX - nst.P1)
    return X, nst


MUTATIONS["admm_step"] = _admm_dual_sign


def _mut_objective_terms(X, Yl, Yh, pr, omega=None):   # lambda1 dropped from the Y_h term
    a, b, c = _orig["objective_terms"](X, Yl, Yh, pr, omega)
    return a, b / pr.lam1, c


def _mut_primal_residuals(X, st, pr):                  # first residual against X, not B X
    r1 = X - st.P1
    r2 = X - st.P2
    return float(np.sqrt(np.sum(r1 * r1))), float(np.sqrt(np.sum(r2 * r2)))


def _mut_fused_denominator(p, q, window, K):             # the patch factor |P| dropped
    return _orig["fused_denominator"](p, q, window, 0)


def _mut_aliasing_groups(p, q, d):                      # aliases along one axis only
    rows, cols = _orig["aliasing_groups"](p, q, d)
    return rows, np.repeat(cols[:, :1], cols.shape[1], axis=1)


def _mut_upsample(Yl, d):                              # upsample shifted by one pixel
    return np.roll(_orig["upsample_nn"](Yl, d), 1, axis=-1)


def _mut_initial_state(Yl, pr, init="upsample"):       # P1 started at X0 instead of B X0
    X0, st = _orig["initial_state"](Yl, pr, init)
    st.P1 = X0.copy()
    return X0, st


MUTATIONS["upsample_nn"] = _mut_upsample
MUTATIONS["initial_state"] = _mut_initial_state
MUTATIONS["objective_terms"] = _mut_objective_terms
MUTATIONS["fused_denominator"] = _mut_fused_denominator
MUTATIONS["aliasing_groups"] = _mut_aliasing_groups
MUTATIONS["primal_residuals"] = _mut_primal_residuals


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, monkeypatch):
    monkeypatch.setattr(o, name, MUTATIONS[name])
    failures = 0
    for pin in FAST_PINS:
        try:
            pin()
        except AssertionError:
            failures += 1
        except Exception:             # a crash under the mutation also counts as caught
            failures += 1
    assert failures >= 1, f"no pin caught the planted mistake in {name}"
