"""Planted mistakes in the oracle must be caught by its pins.

Each case monkeypatches one oracle function with a plausible slip (a dropped
term, a flipped sign, a wrong index or factor) and checks that at least one
pin of tests/test_oracle.py or tests/test_oracle_iterates.py fails.  All on
the CPU.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import admm, pgd, wls
from tests import test_oracle as T
from tests import test_oracle_iterates as TI


def _must_fail(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_dropped_factor_two_in_gradient(monkeypatch):
    orig = wls.scenario_gradient
    monkeypatch.setattr(wls, "scenario_gradient", lambda W, s, x: 0.5 * orig(W, s, x))
    _must_fail(T.test_objective_and_gradient_hand_values)


def test_missing_scenario_probability_in_objective(monkeypatch):
    def f_s(W, s, x):
        r = W.A[s] @ x - W.p
        return float(np.sum(W.w * r * r))
    monkeypatch.setattr(wls, "scenario_objective", f_s)
    _must_fail(T.test_objective_and_gradient_hand_values)


def test_transposed_operand_in_gradient(monkeypatch):
    def g_s(W, s, x):
        r = W.A[s] @ x - W.p
        # weights applied on the wrong side of the product
        return 2.0 * W.c[s] * (W.A[s].T @ r) * np.mean(W.w)
    monkeypatch.setattr(wls, "scenario_gradient", g_s)
    _must_fail(T.test_objective_and_gradient_hand_values)


def test_wrong_sign_of_dual_in_rhs(monkeypatch):
    def rhs(self, s, z, y_s):
        return self.b[s] + 0.5 * self.rho * (z + y_s / self.rho)
    monkeypatch.setattr(admm.AdmmSetup, "rhs", rhs)
    _must_fail(T.test_x_update_hand_value)


def test_flipped_bb_sign(monkeypatch):
    orig = admm.bb_step
    monkeypatch.setattr(admm, "bb_step", lambda d, dp, y, yp: -orig(d, dp, y, yp))
    _must_fail(T.test_bb_step_hand_values)


def test_z_update_without_dual_term(monkeypatch):
    monkeypatch.setattr(admm, "z_update", lambda W, x, y, rho, z_mode=0: wls.project(W, np.mean(x, axis=0)))
    _must_fail(T.test_admm_bb_reaches_brute_force, 100)


def test_tolerance_with_n_instead_of_sqrt_n(monkeypatch):
    def tol(x, z, y, ea, er):
        N, n = x.shape
        base = ea * math.sqrt(N * n)
        return base + er * max(float(np.linalg.norm(x)), N * float(np.linalg.norm(z))), base + er * float(np.linalg.norm(y))
    monkeypatch.setattr(admm, "tolerances", tol)
    _must_fail(T.test_residuals_and_tolerances_hand_values)


def test_residual_dual_without_sqrt_n(monkeypatch):
    def res(x, z, z_old, rho):
        return float(np.linalg.norm(x - z[None, :])), rho * float(np.linalg.norm(z - z_old))
    monkeypatch.setattr(admm, "residuals", res)
    _must_fail(T.test_residuals_and_tolerances_hand_values)


# ---- pins of the ADMM-BB iterates (tests/test_oracle_iterates.py) ----

@pytest.fixture(scope="module")
def tiny_w():
    return TI.tiny_problem()


def test_full_rho_in_rhs_breaks_subproblem_minimality(monkeypatch, tiny_w):
    def rhs(self, s, z, y_s):
        return self.b[s] + self.rho * (z - y_s / self.rho)
    monkeypatch.setattr(admm.AdmmSetup, "rhs", rhs)
    _must_fail(TI.test_every_x_update_minimises_its_subproblem, tiny_w, False)


def test_rhs_without_scenario_probability_breaks_subproblem_minimality(monkeypatch, tiny_w):
    def rhs(self, s, z, y_s):
        return self.b[s] / self.W.c[s] + 0.5 * self.rho * (z - y_s / self.rho)
    monkeypatch.setattr(admm.AdmmSetup, "rhs", rhs)
    _must_fail(TI.test_every_x_update_minimises_its_subproblem, tiny_w, False)


def test_z_update_without_dual_term_breaks_dual_feasibility(monkeypatch, tiny_w):
    # z itself barely moves (sum_s y_s vanishes off the active bounds, where the
    # two forms agree); the duals it leaves behind leave the normal cone
    monkeypatch.setattr(admm, "z_update", lambda W, x, y, rho, z_mode=0: wls.project(W, np.mean(x, axis=0)))
    _must_fail(TI.test_fixed_step_duals_are_dual_feasible_for_the_z_step, tiny_w)


def test_z_update_with_dual_times_rho_breaks_dual_feasibility(monkeypatch, tiny_w):
    monkeypatch.setattr(admm, "z_update",
                        lambda W, x, y, rho, z_mode=0: wls.project(W, np.mean(x + y * rho, axis=0)))
    _must_fail(TI.test_fixed_step_duals_are_dual_feasible_for_the_z_step, tiny_w)


def test_step_always_rho_breaks_the_sign_rule(monkeypatch, tiny_w):
    monkeypatch.setattr(admm, "choose_tau", lambda beta, rho, bb_clamp=0.0: rho)
    _must_fail(TI.test_bb_value_is_the_least_squares_secant_fit_and_follows_the_sign_rule, tiny_w)


def test_bb_with_swapped_dual_difference_breaks_the_secant_fit(monkeypatch, tiny_w):
    orig = admm.bb_step
    monkeypatch.setattr(admm, "bb_step", lambda d, dp, y, yp: orig(d, dp, yp, y))
    _must_fail(TI.test_bb_value_is_the_least_squares_secant_fit_and_follows_the_sign_rule, tiny_w)


def test_dual_sign_flip_moves_the_fixed_point(monkeypatch, tiny_w):
    # y_s enters the right-hand side with the wrong sign: the optimum with its
    # duals is no longer a fixed point
    def rhs(self, s, z, y_s):
        return self.b[s] + 0.5 * self.rho * (z + y_s / self.rho)
    monkeypatch.setattr(admm.AdmmSetup, "rhs", rhs)
    _must_fail(TI.test_the_optimum_with_its_duals_is_a_fixed_point, tiny_w, 0)


# ---- pins of the operators, the PGD step bound and the penalty default ----

def test_normal_apply_without_scenario_probability(monkeypatch):
    def na(W, s, v, rho):
        v = np.asarray(v, dtype=np.float64)
        return W.A[s].T @ (W.w * (W.A[s] @ v)) + 0.5 * rho * v
    monkeypatch.setattr(wls, "normal_apply", na)
    _must_fail(T.test_operator_hand_values)


def test_normal_apply_with_full_rho_shift(monkeypatch):
    def na(W, s, v, rho):
        v = np.asarray(v, dtype=np.float64)
        return W.A[s].T @ (W.c[s] * W.w * (W.A[s] @ v)) + rho * v
    monkeypatch.setattr(wls, "normal_apply", na)
    _must_fail(T.test_operator_hand_values)


def test_normal_apply_without_shift_breaks_gradient_identity(monkeypatch):
    def na(W, s, v, rho):
        v = np.asarray(v, dtype=np.float64)
        return W.A[s].T @ (W.c[s] * W.w * (W.A[s] @ v))
    monkeypatch.setattr(wls, "normal_apply", na)
    W = wls.from_problem(__import__("synth").make_tiny(0))
    _must_fail(T.test_normal_operator_is_the_subproblem_gradient, W)


def test_normal_scale_without_absolute_values(monkeypatch):
    monkeypatch.setattr(wls, "normal_apply_abs", lambda W, s, v, rho: wls.normal_apply(W, s, v, rho))
    _must_fail(T.test_operator_hand_values)


def test_transpose_scale_without_absolute_values(monkeypatch):
    monkeypatch.setattr(wls, "rmatvec_abs", lambda W, s, t: wls.rmatvec(W, s, t))
    _must_fail(T.test_operator_hand_values)


def test_hessian_without_factor_two(monkeypatch):
    orig = pgd.hessian_apply
    monkeypatch.setattr(pgd, "hessian_apply", lambda W, v: 0.5 * orig(W, v))
    _must_fail(T.test_operator_hand_values)
    _must_fail(T.test_lipschitz_is_the_closed_form_largest_eigenvalue)


def test_lipschitz_with_too_few_power_steps(monkeypatch):
    orig = pgd.lipschitz
    monkeypatch.setattr(pgd, "lipschitz", lambda W, iters=30, seed=0: orig(W, iters=2))
    _must_fail(T.test_lipschitz_is_the_closed_form_largest_eigenvalue)


def test_default_rho_without_factor_two(monkeypatch):
    monkeypatch.setattr(wls, "default_rho", lambda W, scale=1.0: scale * wls.mean_gram_diagonal(W))
    _must_fail(T.test_operator_hand_values)


def test_gram_diagonal_without_weights(monkeypatch):
    def mgd(W):
        return float(np.mean([np.mean(np.asarray(W.A[s].multiply(W.A[s]).sum(axis=0)).ravel()) for s in range(W.N)]))
    monkeypatch.setattr(wls, "mean_gram_diagonal", mgd)
    _must_fail(T.test_operator_hand_values)
