"""Planted mistakes in the oracle must be caught by its pins.

Each case monkeypatches one oracle function with a plausible slip (a dropped
term, a flipped sign, a wrong index or factor) and checks that at least one
pin of tests/test_oracle.py fails.  All on the CPU.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import admm, wls
from tests import test_oracle as T


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
