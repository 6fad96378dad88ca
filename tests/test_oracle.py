"""CPU pins of the FP64 oracle against facts that do not come from the oracle.

Each test names what pins it: hand-worked values of the paper's formulas
(tests/golden/admm_steps.json), closed forms, brute-force enumeration,
scipy's bounded least-squares solver, finite differences and invariances of
the problem of Sec. 2.1.
"""
from __future__ import annotations

import math

import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp

import synth
from oracle import admm, exact, pgd, wls
from tests import _helpers as H


# ----------------------------------------------------------------------------
# formulas against hand-worked values
# ----------------------------------------------------------------------------

def test_objective_and_gradient_hand_values():
    g = H.golden("admm_steps.json")["objective"]
    for ckey, fkey, gkey in (("c_equal", "f_equal", "grad_equal"), ("c_weighted", "f_weighted", "grad_weighted")):
        P = H.problem_from_dense(g["A"], g["w"], g["p"], c=g[ckey])
        W = wls.from_problem(P)
        x = np.asarray(g["x"])
        assert wls.objective(W, x) == pytest.approx(g[fkey], rel=1e-15)
        np.testing.assert_allclose(wls.gradient(W, x), g[gkey], rtol=1e-15)


def test_x_update_hand_value():
    g = H.golden("admm_steps.json")["x_update"]
    P = H.problem_from_dense([g["A"]], g["w"], g["p"])
    W = wls.from_problem(P)
    S = admm.AdmmSetup(W, g["rho"])
    x = S.x_update(0, np.asarray(g["z"]), np.asarray(g["y"]))
    np.testing.assert_allclose(x, g["x"], rtol=1e-14)


def test_z_update_hand_values():
    g = H.golden("admm_steps.json")["z_update"]
    P = H.problem_from_dense([np.ones((1, 3))], [1.0], [0.0], lb=g["lb"], ub=g["ub"])
    W = wls.from_problem(P)
    x, y = np.asarray(g["x"]), np.asarray(g["y"])
    np.testing.assert_allclose(admm.z_update(W, x, y, g["rho"], 0), g["z_mode0"], rtol=1e-15)
    np.testing.assert_allclose(admm.z_update(W, x, y, g["rho"], 1), g["z_mode1"], rtol=1e-15)


def test_bb_step_hand_values():
    g = H.golden("admm_steps.json")["bb_step"]
    d, dp, yp = (np.asarray(g[k]) for k in ("d", "d_prev", "y_prev"))
    for sfx in ("pos", "neg"):
        beta = admm.bb_step(d, dp, np.asarray(g["y_" + sfx]), yp)
        assert beta == pytest.approx(g["beta_" + sfx], rel=1e-15)
        assert admm.choose_tau(beta, g["rho"]) == pytest.approx(g["tau_" + sfx], rel=1e-15)
    assert math.isnan(admm.bb_step(d, d, yp, yp))
    assert admm.choose_tau(float("nan"), 3.0) == 3.0
    assert admm.choose_tau(100.0, 3.0, bb_clamp=10.0) == 30.0


def test_residuals_and_tolerances_hand_values():
    g = H.golden("admm_steps.json")["residuals"]
    x, z, zo, y = (np.asarray(g[k]) for k in ("x", "z", "z_old", "y"))
    rp, rd = admm.residuals(x, z, zo, g["rho"])
    assert rp == pytest.approx(g["r_prim"], rel=1e-15)
    assert rd == pytest.approx(g["r_dual"], rel=1e-15)
    ep, ed = admm.tolerances(x, z, y, g["eps_abs"], g["eps_rel"])
    assert ep == pytest.approx(g["eps_prim"], rel=1e-14)
    assert ed == pytest.approx(g["eps_dual"], rel=1e-14)


# ----------------------------------------------------------------------------
# objective, gradient and normal equations on generated problems
# ----------------------------------------------------------------------------

@pytest.fixture(scope="module")
def tiny():
    return synth.make_tiny(0)


@pytest.fixture(scope="module")
def tinyW(tiny):
    return wls.from_problem(tiny)


@pytest.fixture(scope="module")
def tinyQ(tinyW):
    return wls.quadratic_form(tinyW)


def test_objective_equals_quadratic_form(tinyW, tinyQ):
    Hm, g0, const = tinyQ
    rng = np.random.default_rng(1)
    for _ in range(3):
        x = rng.uniform(0, 2, tinyW.n)
        f1 = wls.objective(tinyW, x)
        f2 = wls.objective_quadratic(Hm, g0, const, x)
        assert f1 == pytest.approx(f2, rel=1e-11)
        np.testing.assert_allclose(wls.gradient(tinyW, x), Hm @ x - g0, rtol=1e-10, atol=1e-10 * np.abs(g0).max())


def test_gradient_central_differences(tinyW):
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, tinyW.n)
    g = wls.gradient(tinyW, x)
    for _ in range(4):
        d = rng.normal(size=tinyW.n)
        h = 1e-4
        fd = (wls.objective(tinyW, x + h * d) - wls.objective(tinyW, x - h * d)) / (2 * h)
        # f is quadratic: central differences are exact up to rounding
        assert fd == pytest.approx(g @ d, rel=1e-7)


def test_x_update_solves_subproblem(tinyW):
    """x_update minimises f_s(x) + rho/2 ||x - z + y/rho||^2 (Sec. 2.2): its gradient
    2 A^T diag(c w)(A x - p) + rho (x - z + y/rho) vanishes."""
    rho = wls.default_rho(tinyW)
    S = admm.AdmmSetup(tinyW, rho)
    rng = np.random.default_rng(3)
    z = rng.uniform(0, 1, tinyW.n)
    y = rng.normal(size=tinyW.n)
    for s in range(tinyW.N):
        x = S.x_update(s, z, y)
        grad = wls.scenario_gradient(tinyW, s, x) + rho * (x - z + y / rho)
        scale = np.abs(wls.scenario_gradient(tinyW, s, np.zeros(tinyW.n))).max() + rho * np.abs(z).max()
        assert np.abs(grad).max() <= 1e-9 * scale


def test_spmv_references_match_dense(tinyW):
    rng = np.random.default_rng(4)
    v = rng.normal(size=tinyW.n)
    t = rng.normal(size=tinyW.m)
    D = tinyW.A[1].toarray()
    np.testing.assert_allclose(wls.matvec(tinyW, 1, v), D @ v, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(wls.rmatvec(tinyW, 1, t), D.T @ t, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(wls.matvec_abs(tinyW, 1, v), np.abs(D) @ np.abs(v), rtol=1e-13)


# ----------------------------------------------------------------------------
# operators of the x-update, PGD step size and penalty default
# ----------------------------------------------------------------------------

def _operator_case():
    g = H.golden("admm_steps.json")["operators"]
    P = H.problem_from_dense(g["A"], g["w"], g["p"], c=g["c"])
    return g, wls.from_problem(P)


def test_operator_hand_values():
    """B_s v (Appendix A), its |.| scale, |A_s|^T |t|, H v, the Gram diagonal
    mean and the default penalty against values worked by hand."""
    g, W = _operator_case()
    v, t, rho = np.asarray(g["v"]), np.asarray(g["t"]), g["rho"]
    for s in range(W.N):
        np.testing.assert_allclose(wls.normal_apply(W, s, v, rho), g["normal"][s], rtol=1e-15)
        np.testing.assert_allclose(wls.normal_apply_abs(W, s, v, rho), g["normal_abs"][s], rtol=1e-15)
        np.testing.assert_allclose(wls.rmatvec_abs(W, s, t), g["rmatvec_abs"][s], rtol=1e-15)
    np.testing.assert_allclose(pgd.hessian_apply(W, v), g["hessian_v"], rtol=1e-15)
    assert wls.mean_gram_diagonal(W) == pytest.approx(g["mean_gram_diagonal"], rel=1e-15)
    assert wls.default_rho(W) == pytest.approx(g["default_rho"], rel=1e-15)


def test_lipschitz_is_the_closed_form_largest_eigenvalue():
    """Power iteration on the hand-worked 2 x 2 Hessian [[24, 8], [8, 17]]
    reaches lambda_max = (41 + sqrt(305)) / 2 (eigenvalue ratio 0.4, 30 steps)."""
    g, W = _operator_case()
    assert pgd.lipschitz(W) == pytest.approx((41.0 + math.sqrt(305.0)) / 2.0, rel=1e-10)


def test_lipschitz_matches_eigvalsh(tinyW, tinyQ):
    """The step-size bound of Sec. 2.1's PGD against LAPACK's symmetric
    eigenvalues of the quadratic form's Hessian (itself pinned by the objective
    identity); a unit-norm power iterate never overshoots lambda_max."""
    Hm = tinyQ[0]
    lam = np.linalg.eigvalsh(Hm)[-1]
    L = pgd.lipschitz(tinyW)
    assert L <= lam * (1 + 1e-12)
    assert L == pytest.approx(lam, rel=1e-6)


def test_normal_operator_is_the_subproblem_gradient(tinyW):
    """grad f_s(v) - grad f_s(0) = 2 A_s^T diag(c_s w) A_s v (Sec. 2.1; the
    gradient is pinned by central differences), so B_s v equals half of it
    plus rho/2 v, and H v is the sum of those differences."""
    rng = np.random.default_rng(5)
    rho = 0.7
    v = rng.normal(size=tinyW.n)
    zero = np.zeros(tinyW.n)
    hv = np.zeros(tinyW.n)
    for s in range(tinyW.N):
        dg = wls.scenario_gradient(tinyW, s, v) - wls.scenario_gradient(tinyW, s, zero)
        scale = np.abs(dg).max()
        np.testing.assert_allclose(wls.normal_apply(tinyW, s, v, rho), 0.5 * dg + 0.5 * rho * v,
                                   rtol=0, atol=1e-12 * scale)
        hv += dg
    np.testing.assert_allclose(pgd.hessian_apply(tinyW, v), hv, rtol=0, atol=1e-12 * np.abs(hv).max())


def test_absolute_scales_bound_the_products(tinyW):
    """|B_s v| <= (|A_s|^T c_s W |A_s| + rho/2) |v| and |A_s^T t| <= |A_s|^T |t|
    entry by entry (triangle inequality), with equality for nonnegative
    arguments because A_s >= 0 (Sec. 2.1)."""
    rng = np.random.default_rng(6)
    rho = 0.3
    v = rng.normal(size=tinyW.n)
    t = rng.normal(size=tinyW.m)
    for s in range(tinyW.N):
        nb = wls.normal_apply_abs(tinyW, s, v, rho)
        assert np.all(np.abs(wls.normal_apply(tinyW, s, v, rho)) <= nb * (1 + 1e-13))
        np.testing.assert_allclose(nb, wls.normal_apply(tinyW, s, np.abs(v), rho), rtol=1e-13)
        rb = wls.rmatvec_abs(tinyW, s, t)
        assert np.all(np.abs(wls.rmatvec(tinyW, s, t)) <= rb * (1 + 1e-13))
        np.testing.assert_allclose(rb, wls.rmatvec(tinyW, s, np.abs(t)), rtol=1e-13)
        # mixed signs make the scale strictly larger somewhere
        assert np.any(nb > np.abs(wls.normal_apply(tinyW, s, v, rho)) * (1 + 1e-6))


def test_gram_diagonal_from_second_differences(tinyW):
    """(G_s)_jj is half the second derivative of f_s along spot j (Sec. 2.1):
    f_s(h e_j) + f_s(-h e_j) - 2 f_s(0) = 2 h^2 (G_s)_jj exactly for a
    quadratic; the penalty default is twice the mean over s and j."""
    h = 0.5
    tot = 0.0
    f0 = [wls.scenario_objective(tinyW, s, np.zeros(tinyW.n)) for s in range(tinyW.N)]
    for s in range(tinyW.N):
        d = np.empty(tinyW.n)
        for j in range(tinyW.n):
            e = np.zeros(tinyW.n)
            e[j] = h
            d[j] = (wls.scenario_objective(tinyW, s, e) + wls.scenario_objective(tinyW, s, -e) - 2 * f0[s]) / (2 * h * h)
        tot += d.mean()
    mean_diag = tot / tinyW.N
    assert wls.mean_gram_diagonal(tinyW) == pytest.approx(mean_diag, rel=1e-9)
    assert wls.default_rho(tinyW) == pytest.approx(2.0 * mean_diag, rel=1e-9)
    assert wls.default_rho(tinyW, scale=0.25) == pytest.approx(0.5 * mean_diag, rel=1e-9)


# ----------------------------------------------------------------------------
# exact minimisers: brute force vs a library solver vs the polish
# ----------------------------------------------------------------------------

def _bvls(W: wls.Wls):
    rows, rhs = [], []
    for s in range(W.N):
        sw = np.sqrt(W.c[s] * W.w)
        rows.append(sp.diags(sw) @ W.A[s])
        rhs.append(sw * W.p)
    r = so.lsq_linear(sp.vstack(rows).toarray(), np.concatenate(rhs), bounds=(W.lb, W.ub),
                      method="bvls", tol=1e-15, max_iter=10000)
    return r.x


@pytest.mark.parametrize("seed", [100, 101, 102, 103])
def test_brute_force_matches_bvls_and_active_set(seed):
    P = synth.make_brute(seed)
    W = wls.from_problem(P)
    Hm, g0, _ = wls.quadratic_form(W)
    xb, labels, unique = exact.brute_force(Hm, g0, W.lb, W.ub)
    assert unique
    xl = _bvls(W)
    np.testing.assert_allclose(xb, xl, atol=1e-10)
    xa, info = exact.active_set(W, H=Hm, g0=g0)
    assert info["kkt"] <= 1e-12
    np.testing.assert_allclose(xa, xb, atol=1e-10)


def test_active_set_matches_bvls_tiny(tinyW, tinyQ):
    Hm, g0, const = tinyQ
    xa, info = exact.active_set(tinyW, H=Hm, g0=g0)
    assert info["kkt"] <= 1e-12
    xl = _bvls(tinyW)
    fa = wls.objective(tinyW, xa)
    fl = wls.objective(tinyW, xl)
    assert fa <= fl * (1 + 1e-12)
    assert fa == pytest.approx(fl, rel=1e-10)


def test_planted_interior_solution():
    """N = 1 and p = A x_true with x_true inside the box: f* = 0, x* = x_true."""
    P = synth.make_brute(104)
    P1 = P.subset([0])
    rng = np.random.default_rng(5)
    x_true = rng.uniform(0.1, 0.9, P.n) * P.ub
    W0 = wls.from_problem(P1)
    p = W0.A[0] @ x_true
    W = wls.from_problem(H.with_presc(P1, p))
    res = admm.admm_bb(W, eps_abs=1e-13, eps_rel=1e-13, obj_rel_tol=0.0, max_iter=20000)
    assert res.converged
    np.testing.assert_allclose(res.z, x_true, rtol=1e-6, atol=1e-8)
    assert wls.objective(W, res.z) <= 1e-12 * float(W.p @ W.p)


def test_interior_optimum_is_normal_equation_solution():
    """With the box inactive, x* = H^{-1} g0 (unconstrained closed form)."""
    P = synth.make_brute(105)
    W = wls.from_problem(P)
    Hm, g0, _ = wls.quadratic_form(W)
    xu = np.linalg.solve(Hm, g0)
    Wb = wls.Wls(A=W.A, c=W.c, w=W.w, p=W.p, lb=np.full(W.n, -1e6), ub=np.full(W.n, 1e6))
    xa, info = exact.active_set(Wb, H=Hm, g0=g0)
    np.testing.assert_allclose(xa, xu, rtol=1e-9)
    res = admm.admm_bb(Wb, eps_abs=1e-12, eps_rel=1e-12, obj_rel_tol=0.0, max_iter=20000)
    np.testing.assert_allclose(res.z, xu, rtol=1e-7)


# ----------------------------------------------------------------------------
# invariances of the problem
# ----------------------------------------------------------------------------

def _xstar(P):
    W = wls.from_problem(P)
    Hm, g0, _ = wls.quadratic_form(W)
    x, info = exact.active_set(W, H=Hm, g0=g0)
    assert info["kkt"] <= 1e-12
    return x, wls.objective(W, x)


def test_identical_scenarios_scale_objective():
    P = synth.make_brute(106).subset([0])
    x1, f1 = _xstar(P)
    P3 = H.duplicate_scenario(H.duplicate_scenario(P, 0), 0)
    x3, f3 = _xstar(P3)
    np.testing.assert_allclose(x3, x1, atol=1e-10)
    assert f3 == pytest.approx(3 * f1, rel=1e-12)


def test_probability_two_equals_duplicated_scenario():
    """Sec. 2.1: w~_{s,i} = c_s w_i, so c_s = 2 is the same problem as scenario s twice."""
    P = synth.make_brute(107)
    xa, fa = _xstar(H.scaled_prob(P, 1, 2.0))
    xb, fb = _xstar(H.duplicate_scenario(P, 1))
    np.testing.assert_allclose(xa, xb, atol=1e-10)
    assert fa == pytest.approx(fb, rel=1e-12)


def test_weight_scaling_invariance():
    P = synth.make_brute(108)
    x1, f1 = _xstar(P)
    x2, f2 = _xstar(H.with_weights(P, 3.5 * P.struct_weight))
    np.testing.assert_allclose(x2, x1, atol=1e-10)
    assert f2 == pytest.approx(3.5 * f1, rel=1e-12)


# ----------------------------------------------------------------------------
# ADMM-BB and PGD reach the exact minimiser
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [100, 102, 103])
def test_admm_bb_reaches_brute_force(seed):
    P = synth.make_brute(seed)
    W = wls.from_problem(P)
    Hm, g0, _ = wls.quadratic_form(W)
    xb, _, _ = exact.brute_force(Hm, g0, W.lb, W.ub)
    res = admm.admm_bb(W, eps_abs=1e-12, eps_rel=1e-12, obj_rel_tol=0.0, max_iter=50000)
    assert res.converged
    assert wls.kkt_residual(W, res.z) <= 1e-10
    np.testing.assert_allclose(res.z, xb, atol=1e-9)


def test_admm_bb_and_pgd_agree_tiny(tinyW, tinyQ):
    Hm, g0, const = tinyQ
    xa, _ = exact.active_set(tinyW, H=Hm, g0=g0)
    fstar = wls.objective(tinyW, xa)
    res = admm.admm_bb(tinyW, rho=wls.default_rho(tinyW, 0.125), eps_abs=1e-12, eps_rel=1e-12,
                       obj_rel_tol=0.0, max_iter=20000)
    assert wls.kkt_residual(tinyW, res.z) <= 1e-10
    q = pgd.pgd_armijo(tinyW, obj_rel_tol=1e-15, max_iter=20000)
    assert res.obj == pytest.approx(fstar, rel=1e-10)
    assert q.obj == pytest.approx(res.obj, rel=1e-8)


def test_admm_default_stop_reaches_objective_tolerance(tinyW, tinyQ):
    """With the paper's settings (eps_abs = eps_rel = 1e-6 combined with a 1e-5
    relative objective change, Sec. 2.3) the returned z is within 1e-5 of f*."""
    Hm, g0, const = tinyQ
    xa, _ = exact.active_set(tinyW, H=Hm, g0=g0)
    fstar = wls.objective(tinyW, xa)
    res = admm.admm_bb(tinyW, max_iter=20000)
    assert res.converged
    assert (res.obj - fstar) / fstar <= 1e-5


def test_pgd_objective_monotone(tinyW):
    q = pgd.pgd_armijo(tinyW, max_iter=300)
    f = [h["obj"] for h in q.history]
    assert all(b <= a for a, b in zip(f, f[1:]))


def test_paper_literal_z_update_can_miss_kkt():
    """Reading of Sec. 2.2 step 2: the printed z = max(mean x_s, 0) drops the
    y_s/rho term of consensus ADMM; on these instances its fixed point is not a
    minimiser while the consensus form's is."""
    misses = 0
    for seed in (100, 101):
        W = wls.from_problem(synth.make_brute(seed))
        r0 = admm.admm_bb(W, eps_abs=1e-12, eps_rel=1e-12, obj_rel_tol=0.0, max_iter=20000, z_mode=0)
        r1 = admm.admm_bb(W, eps_abs=1e-12, eps_rel=1e-12, obj_rel_tol=0.0, max_iter=20000, z_mode=1)
        assert wls.kkt_residual(W, r0.z) <= 1e-10
        misses += wls.kkt_residual(W, r1.z) > 1e-6
    assert misses >= 1
