"""ADMM-BB for the consensus form of the robust problem (FP64, CPU).

Test infrastructure (see the package docstring): never imported by the product.

Follows Sec. 2.2 and Appendix A in order:

  setup      For every scenario form B_s = A~_s^T A~_s + (rho/2) I with
             A~_s = diag(sqrt(c_s w)) A_s, factor it once by Cholesky and keep
             the factor (App. A); keep b_s = A~_s^T p~ = A_s^T diag(c_s w) p.
  x-update   Each scenario solves the regularised WLS subproblem of Sec. 2.2
             through its normal equations B_s x_s = c_s,
             c_s = b_s + (rho/2)(z - y_s/rho)   (App. A), two triangular solves.
  z-update   z = P( mean_s (x_s + y_s/rho) )  (consensus form, default) or the
             form printed in Sec. 2.2, z = P( mean_s x_s )  (z_mode=1).
  BB step    beta = -<dd, dy> / ||dd||^2 with dy = y^k - y^{k-1} and
             dd = (x^{k+1} - z^{k+1}) - (x^k - z^k) over the stacked vectors;
             beta replaces rho in the dual update when positive (Sec. 2.2, BB).
  y-update   y_s += tau (x_s - z)  with tau = beta or rho  (Sec. 2.2).
  stop       ||r_prim|| <= eps_prim and ||r_dual|| <= eps_dual with the
             eps_abs / eps_rel tolerances of Sec. 2.2, combined (AND) with a
             relative objective change <= obj_rel_tol (Sec. 2.3); returns z.

Readings where the paper is silent or garbled (all listed in the design notes):
the consensus z-update keeps the y/rho term that Sec. 2.2 drops; the BB
scalar is global over the stacked vectors; at the first iteration, or when
||dd|| = 0 or beta is not finite, tau = rho; z0 = 0, y0 = 0, x_s = z0 at start;
the combined stop is an AND; the objective is evaluated at the feasible z.

Parity: the end point is pinned by brute force, closed forms and the active-set
polish; the paper prints no iterate, so the iterates are pinned by what its
statement fixes (tests/test_oracle_iterates.py): every x_s minimises the
subproblem of Sec. 2.2, every z minimises the augmented Lagrangian over the
box, every BB step is the least-squares secant fit of Delta y by Delta d, a
one-scenario problem follows its closed-form geometric trajectory, and the
optimal (z*, y*) is a fixed point.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from . import wls


@dataclasses.dataclass
class AdmmResult:
    z: np.ndarray
    x: np.ndarray            # stacked N x n
    y: np.ndarray            # stacked N x n
    iters: int
    converged: bool
    obj: float
    history: List[dict]
    rho: float


class AdmmSetup:
    """Cached per-scenario Cholesky factors and right-hand-side constants."""

    def __init__(self, W: wls.Wls, rho: float):
        self.W = W
        self.rho = float(rho)
        n = W.n
        self.factors = []
        self.b = np.zeros((W.N, n))
        for s in range(W.N):
            B = wls.scenario_gram(W, s) + 0.5 * self.rho * np.eye(n)
            self.factors.append(sla.cho_factor(B, lower=True, check_finite=False))
            self.b[s] = W.A[s].T @ (W.c[s] * W.w * W.p)

    def rhs(self, s: int, z: np.ndarray, y_s: np.ndarray) -> np.ndarray:
        """c_s = b_s + (rho/2)(z - y_s/rho)   (App. A)."""
        return self.b[s] + 0.5 * self.rho * (z - y_s / self.rho)

    def x_update(self, s: int, z: np.ndarray, y_s: np.ndarray) -> np.ndarray:
        """Solve B_s x = c_s with the cached factor (forward then back substitution)."""
        return sla.cho_solve(self.factors[s], self.rhs(s, z, y_s), check_finite=False)


def z_update(W: wls.Wls, x: np.ndarray, y: np.ndarray, rho: float, z_mode: int = 0) -> np.ndarray:
    """z = P(mean_s(x_s + y_s/rho))  (z_mode 0)  or  P(mean_s x_s)  (z_mode 1, as printed)."""
    if z_mode == 0:
        avg = np.mean(x + y / rho, axis=0)
    else:
        avg = np.mean(x, axis=0)
    return wls.project(W, avg)


def bb_step(d: np.ndarray, d_prev: np.ndarray, y: np.ndarray, y_prev: np.ndarray) -> float:
    """beta = -<dd, dy> / ||dd||^2, dd = d - d_prev, dy = y - y_prev (stacked); nan when ||dd|| = 0."""
    dd = (d - d_prev).ravel()
    dy = (y - y_prev).ravel()
    nd = float(dd @ dd)
    if nd == 0.0:
        return float("nan")
    return -float(dd @ dy) / nd


def choose_tau(beta: float, rho: float, bb_clamp: float = 0.0) -> float:
    """Use beta in place of rho when beta > 0 (and finite); optional clamp to [rho/c, rho*c]."""
    tau = beta if (math.isfinite(beta) and beta > 0.0) else rho
    if bb_clamp > 0.0:
        tau = min(max(tau, rho / bb_clamp), rho * bb_clamp)
    return tau


def tolerances(x: np.ndarray, z: np.ndarray, y: np.ndarray, eps_abs: float, eps_rel: float):
    """eps_prim = eps_abs sqrt(Nn) + eps_rel max(||x||, sqrt(N)||z||);
    eps_dual = eps_abs sqrt(Nn) + eps_rel ||y||   (Sec. 2.2, stopping criterion)."""
    N, n = x.shape
    base = eps_abs * math.sqrt(N * n)
    ep = base + eps_rel * max(float(np.linalg.norm(x)), math.sqrt(N) * float(np.linalg.norm(z)))
    ed = base + eps_rel * float(np.linalg.norm(y))
    return ep, ed


def residuals(x: np.ndarray, z: np.ndarray, z_old: np.ndarray, rho: float):
    """||r_prim|| = ||(x_1 - z, ..., x_N - z)||, ||r_dual|| = ||(rho(z - z_old), ... N times)||."""
    N = x.shape[0]
    rp = float(np.linalg.norm(x - z[None, :]))
    rd = math.sqrt(N) * rho * float(np.linalg.norm(z - z_old))
    return rp, rd


def admm_bb(W: wls.Wls, rho: Optional[float] = None, eps_abs: float = 1e-6, eps_rel: float = 1e-6,
            obj_rel_tol: float = 1e-5, max_iter: int = 5000, bb: bool = True, z_mode: int = 0,
            bb_clamp: float = 0.0, z0: Optional[np.ndarray] = None, setup: Optional[AdmmSetup] = None,
            record: bool = True, callback=None, y0: Optional[np.ndarray] = None,
            state_callback=None) -> AdmmResult:
    """Run ADMM-BB; returns z and the full iteration history.

    y0: starting duals (N x n, default 0).  state_callback(k, state) receives,
    after iteration k, a dict with z_old, y_old (the values the x-updates used),
    x, z, y (new), tau, beta and d_prev (the previous x - z, None at first)."""
    if setup is None:
        rho = wls.default_rho(W) if (rho is None or rho <= 0) else float(rho)
        setup = AdmmSetup(W, rho)
    rho = setup.rho
    N, n = W.N, W.n
    z = wls.project(W, np.zeros(n) if z0 is None else np.asarray(z0, dtype=np.float64))
    x = np.tile(z, (N, 1))
    y = np.zeros((N, n)) if y0 is None else np.array(y0, dtype=np.float64).reshape(N, n)
    d_prev = None
    y_prev = None
    f_prev = None
    hist = []
    converged = False
    k = 0
    f_k = wls.objective(W, z)
    for k in range(max_iter):
        for s in range(N):
            x[s] = setup.x_update(s, z, y[s])
        z_old = z
        z = z_update(W, x, y, rho, z_mode)
        d = x - z[None, :]
        if bb and d_prev is not None:
            beta = bb_step(d, d_prev, y, y_prev)
            tau = choose_tau(beta, rho, bb_clamp)
        else:
            beta = float("nan")
            tau = rho
        y_prev = y.copy()
        d_before = d_prev
        d_prev = d
        y = y + tau * d
        rp, rd = residuals(x, z, z_old, rho)
        ep, ed = tolerances(x, z, y, eps_abs, eps_rel)
        f_prev = f_k
        f_k = wls.objective(W, z)
        if record:
            hist.append(dict(k=k, obj=f_k, r_prim=rp, r_dual=rd, eps_prim=ep, eps_dual=ed,
                             tau=tau, beta=beta))
        if callback is not None:
            callback(k, z, f_k)
        if state_callback is not None:
            state_callback(k, dict(z_old=z_old, y_old=y_prev, x=x.copy(), z=z, y=y.copy(), tau=tau, beta=beta,
                                   d_prev=d_before))
        obj_ok = True
        if obj_rel_tol > 0.0:
            obj_ok = k >= 1 and abs(f_k - f_prev) <= obj_rel_tol * abs(f_prev)
        if rp <= ep and rd <= ed and obj_ok:
            converged = True
            break
    return AdmmResult(z=z, x=x, y=y, iters=k + 1, converged=converged, obj=f_k, history=hist, rho=rho)
