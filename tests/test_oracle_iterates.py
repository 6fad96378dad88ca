"""Pins of the oracle's ADMM-BB iterates (Sec. 2.2) by what the paper's
statement of the method fixes, not by re-deriving its update formulas:

  * each x_s^{k+1} minimises the subproblem f_s(x) + rho/2 ||x - z^k + y_s^k/rho||^2
    (checked by perturbation: the objective of Sec. 2.1 is pinned separately);
  * each z^{k+1} minimises the augmented Lagrangian over the box,
    sum_s ||x_s^{k+1} - z + y_s^k/rho||^2 (the consensus reading), by perturbation;
  * with the fixed step rho, sum_s y_s^{k+1} lies in the normal cone of the box
    at z^{k+1} (dual feasibility of the z-step, Boyd et al. Sec. 3.3);
  * each BB value is the least-squares secant fit of Delta y by Delta d (the
    1-D quadratic it minimises), and the step follows the paper's sign rule;
  * one scenario, inactive bounds: z^k = z* (1 - r^k) per decoupled spot with
    r = rho / (2 g + rho), the solution of the scalar recurrence;
  * the optimum with its duals y_s* = -grad f_s(z*) is a fixed point.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import admm, exact, wls


def tiny_problem():
    """The tiny workload with unequal scenario probabilities c_s (Sec. 2.1),
    so that every place c_s enters is exercised."""
    P = synth.make_tiny(2)
    W = wls.from_problem(P)
    c = np.linspace(0.5, 1.5, W.N)
    return dataclasses.replace(W, c=c / c.sum())


@pytest.fixture(scope="module")
def tiny():
    return tiny_problem()


def _run_states(W, iters, **kw):
    states = []
    admm.admm_bb(W, max_iter=iters, obj_rel_tol=0.0, eps_abs=0.0, eps_rel=0.0, record=False,
                 state_callback=lambda k, st: states.append(st), **kw)
    return states


def _phi(W, s, x, z, y_s, rho):
    """The subproblem of Sec. 2.2 for scenario s."""
    r = x - z + y_s / rho
    return wls.scenario_objective(W, s, x) + 0.5 * rho * float(r @ r)


@pytest.mark.parametrize("bb", [True, False])
def test_every_x_update_minimises_its_subproblem(tiny, bb):
    W = tiny
    rho = wls.default_rho(W)
    rng = np.random.default_rng(5)
    states = _run_states(W, 12, bb=bb, rho=rho)
    for k in (0, 1, 5, 11):
        st = states[k]
        for s in range(W.N):
            x = st["x"][s]
            base = _phi(W, s, x, st["z_old"], st["y_old"][s], rho)
            scale = max(1.0, float(np.linalg.norm(x)))
            for _ in range(4):
                v = rng.normal(size=W.n)
                v /= np.linalg.norm(v)
                h = 1e-2 * scale
                up = _phi(W, s, x + h * v, st["z_old"], st["y_old"][s], rho)
                dn = _phi(W, s, x - h * v, st["z_old"], st["y_old"][s], rho)
                # strong convexity (Hessian >= rho I) and zero directional derivative
                assert up - base >= 0.45 * rho * h * h
                assert dn - base >= 0.45 * rho * h * h
                assert abs(up - dn) / (2 * h) <= 1e-7 * (abs(base) / scale + rho * scale)


@pytest.mark.parametrize("bb", [True, False])
def test_every_z_update_minimises_the_augmented_lagrangian_over_the_box(tiny, bb):
    W = tiny
    rho = wls.default_rho(W)
    rng = np.random.default_rng(6)
    states = _run_states(W, 12, bb=bb, rho=rho)

    def psi(st, z):
        r = st["x"] - z[None, :] + st["y_old"] / rho
        return float(np.sum(r * r))

    for k in (0, 1, 5, 11):
        st = states[k]
        z = st["z"]
        assert np.all(z >= W.lb) and np.all(z <= W.ub)
        base = psi(st, z)
        for h in (1e-3, 1e-1, 1.0):
            for _ in range(6):
                v = rng.normal(size=W.n)
                zt = wls.project(W, z + h * v)
                assert psi(st, zt) >= base - 1e-12 * max(1.0, base)


def test_fixed_step_duals_are_dual_feasible_for_the_z_step(tiny):
    """With tau = rho, sum_s y_s^{k+1} is in the normal cone of the box at z^{k+1}."""
    W = tiny
    rho = wls.default_rho(W)
    states = _run_states(W, 15, bb=False, rho=rho)
    for st in states:
        z, ysum = st["z"], st["y"].sum(axis=0)
        tol = 1e-9 * (1.0 + float(np.abs(st["y"]).max()))
        free = (z > W.lb) & (z < W.ub)
        at_lb = (z <= W.lb) & ~(z >= W.ub)
        at_ub = (z >= W.ub) & ~(z <= W.lb)
        assert np.all(np.abs(ysum[free]) <= tol)
        assert np.all(ysum[at_lb] <= tol)
        assert np.all(ysum[at_ub] >= -tol)
        assert at_lb.any()  # the tiny problem has active lower bounds: the cone is exercised


def test_bb_value_is_the_least_squares_secant_fit_and_follows_the_sign_rule(tiny):
    W = tiny
    rho = wls.default_rho(W)
    states = _run_states(W, 25, bb=True, rho=rho)
    assert states[0]["tau"] == rho and math.isnan(states[0]["beta"])
    used_bb = 0
    for k in range(1, len(states)):
        st, prev = states[k], states[k - 1]
        dd = (st["x"] - st["z"][None, :]) - st["d_prev"]
        dy = st["y_old"] - prev["y_old"]
        beta = st["beta"]
        assert math.isfinite(beta)

        def fit(b):
            r = dy + b * dd
            return float(np.sum(r * r))

        f0 = fit(beta)
        for dlt in (1e-4, 1e-2, 1.0):
            assert fit(beta * (1 + dlt)) >= f0 * (1 - 1e-12)
            assert fit(beta * (1 - dlt)) >= f0 * (1 - 1e-12)
        assert fit(0.0) >= f0
        # the paper's rule: beta replaces rho only when positive
        assert st["tau"] == (beta if beta > 0 else rho)
        used_bb += beta > 0
    assert used_bb > 0


def _decoupled_one_scenario():
    """One scenario, two spots with disjoint voxel supports (diagonal Gram)."""
    a = np.array([0.8, 0.5, 1.2, 0.3])
    rows, cols = np.arange(4), np.array([0, 0, 1, 1])
    A = sp.csr_matrix((a, (rows, cols)), shape=(4, 2))
    w = np.array([1.0, 0.5, 2.0, 1.0])
    p = np.array([1.0, 0.9, 0.7, 0.6])
    return wls.Wls(A=[A], c=np.array([1.0]), w=w, p=p, lb=np.zeros(2), ub=np.full(2, 100.0))


@pytest.mark.parametrize("z_mode", [0, 1])
def test_one_scenario_follows_the_closed_form_trajectory(z_mode):
    W = _decoupled_one_scenario()
    a, w, p = W.A[0].data, W.w, W.p
    g = np.array([w[0] * a[0] ** 2 + w[1] * a[1] ** 2, w[2] * a[2] ** 2 + w[3] * a[3] ** 2])
    zstar = np.array([w[0] * a[0] * p[0] + w[1] * a[1] * p[1], w[2] * a[2] * p[2] + w[3] * a[3] * p[3]]) / g
    rho = g[0]  # r = 1/3 for the first spot
    zs = []
    admm.admm_bb(W, rho=rho, max_iter=30, obj_rel_tol=0.0, eps_abs=0.0, eps_rel=0.0, z_mode=z_mode,
                 record=False, callback=lambda k, z, f: zs.append(z.copy()))
    r = rho / (2 * g + rho)
    for k, z in enumerate(zs, start=1):
        expect = zstar * (1.0 - r ** k)
        assert np.allclose(z, expect, rtol=1e-12, atol=1e-14), (k, z, expect)


@pytest.mark.parametrize("z_mode", [0, 1])
def test_the_optimum_with_its_duals_is_a_fixed_point(tiny, z_mode):
    W = tiny
    Hm, g0, _ = wls.quadratic_form(W)
    xs, _ = exact.active_set(W, H=Hm, g0=g0)
    y0 = np.stack([-wls.scenario_gradient(W, s, xs) for s in range(W.N)])
    states = _run_states(W, 8, bb=True, z0=xs, y0=y0, z_mode=z_mode)
    scale = float(np.linalg.norm(xs))
    for st in states:
        assert np.linalg.norm(st["z"] - xs) <= 1e-9 * scale
        assert np.linalg.norm(st["x"] - xs[None, :]) <= 1e-9 * scale * math.sqrt(W.N)
        assert np.linalg.norm(st["y"] - y0) <= 1e-9 * max(1.0, float(np.linalg.norm(y0)))
