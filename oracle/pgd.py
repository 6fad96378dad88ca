"""Projected gradient descent with Armijo backtracking (FP64, CPU).

Test infrastructure (see the package docstring): never imported by the product.

Sec. 2.1: from x^0 in the box, each iteration computes grad f(x^k), then tries
step sizes t = alpha, alpha*gamma, alpha*gamma^2, ... until the projected point
x' = P(x^k - t grad f(x^k)) gives sufficient decrease,
    f(x') <= f(x^k) + beta * grad f(x^k)^T (x' - x^k)
(the inequality is printed with the opposite sign in the paper; sufficient
decrease is what the cited Armijo rule means), and stops when the relative
change of the objective falls below a cutoff (Sec. 2.1 and 2.3).
The paper leaves alpha, beta, gamma open; defaults here are alpha = 10/L with
L the largest eigenvalue of the Hessian (power iteration), beta = 1e-4,
gamma = 0.5.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional

import numpy as np

from . import wls


@dataclasses.dataclass
class PgdResult:
    x: np.ndarray
    iters: int
    converged: bool
    obj: float
    history: List[dict]
    alpha: float
    trials: int


def hessian_apply(W: wls.Wls, v: np.ndarray) -> np.ndarray:
    """H v = 2 sum_s A_s^T diag(c_s w) A_s v.  Pinned by a hand-worked value and
    by H v = grad f(v) - grad f(0)."""
    out = np.zeros(W.n)
    for s in range(W.N):
        out += 2.0 * W.c[s] * (W.A[s].T @ (W.w * (W.A[s] @ v)))
    return out


def lipschitz(W: wls.Wls, iters: int = 30, seed: int = 0) -> float:
    """Largest eigenvalue of H by power iteration (deterministic start vector of
    ones).  Pinned by the closed-form eigenvalue of a hand-worked 2 x 2 Hessian
    and by LAPACK's eigenvalues of the quadratic form."""
    v = np.ones(W.n) / np.sqrt(W.n)
    lam = 0.0
    for _ in range(iters):
        hv = hessian_apply(W, v)
        lam = float(np.linalg.norm(hv))
        if lam == 0.0:
            return 0.0
        v = hv / lam
    return lam


def pgd_armijo(W: wls.Wls, alpha: Optional[float] = None, beta: float = 1e-4, gamma: float = 0.5,
               obj_rel_tol: float = 1e-5, kkt_tol: float = 0.0, max_iter: int = 10000,
               max_trials: int = 60, x0: Optional[np.ndarray] = None, record: bool = True) -> PgdResult:
    if alpha is None or alpha <= 0:
        L = lipschitz(W)
        alpha = 10.0 / L if L > 0 else 1.0
    x = wls.project(W, np.zeros(W.n) if x0 is None else np.asarray(x0, dtype=np.float64))
    f = wls.objective(W, x)
    hist = []
    converged = False
    total_trials = 0
    k = 0
    for k in range(max_iter):
        g = wls.gradient(W, x)
        t = alpha
        accepted = False
        for _ in range(max_trials):
            total_trials += 1
            xt = wls.project(W, x - t * g)
            ft = wls.objective(W, xt)
            if ft <= f + beta * float(g @ (xt - x)):
                accepted = True
                break
            t *= gamma
        if not accepted:
            break
        f_old = f
        x, f = xt, ft
        if record:
            hist.append(dict(k=k, obj=f, step=t))
        if kkt_tol > 0.0:
            if wls.kkt_residual(W, x) <= kkt_tol:
                converged = True
                break
        elif abs(f_old - f) <= obj_rel_tol * abs(f_old):
            converged = True
            break
    return PgdResult(x=x, iters=k + 1, converged=converged, obj=f, history=hist, alpha=alpha,
                     trials=total_trials)
