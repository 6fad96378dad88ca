"""Exact minimisers of the box-constrained robust WLS problem (FP64).

Test infrastructure (see the package docstring): never imported by the product.

The problem of Sec. 2.1, min f(x) s.t. lb <= x <= ub, is a convex quadratic
program: f(x) = 1/2 x^T H x - g0^T x + const with H = 2 sum_s A_s^T diag(c_s w) A_s.
Its minimisers are exactly the points satisfying the KKT conditions
   grad_j >= 0 where x_j = lb_j,  grad_j <= 0 where x_j = ub_j,  grad_j = 0 otherwise.
Two independent routes to them live here:

  brute_force     enumerate every labelling of the spots as lower / upper / free
                  (3^n labellings, n <= 12), solve the free block, keep the
                  labelling whose point satisfies KKT.  Slow, no iteration.
  active_set      projected-Newton polish (Bertsekas' projected Newton method
                  for bound-constrained problems): from any start, fix the
                  variables held at a bound by an outward gradient, take the
                  Newton step on the rest, project, backtrack.  Stops when the
                  scaled KKT residual is <= tol.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg as sla

from . import wls


def _chol_solve(M: np.ndarray, b: np.ndarray):
    try:
        c = sla.cho_factor(M, lower=True, check_finite=False)
    except np.linalg.LinAlgError:
        return None
    return sla.cho_solve(c, b, check_finite=False)


def brute_force(H: np.ndarray, g0: np.ndarray, lb: np.ndarray, ub: np.ndarray, slack: float = 1e-12):
    """Return (x, labels, unique) for min 1/2 x^T H x - g0^T x over the box.

    Exhaustive over all 3^n labellings (0 = at lb, 1 = at ub, 2 = free), n <= 12.
    For each free set F the 2^(n-|F|) bound assignments of the other spots are
    solved together (one Cholesky of H_FF, many right-hand sides); a labelling
    survives when its free part lies strictly inside the box and the gradient
    points outward on every bound spot.  With H positive definite exactly one
    labelling survives; `unique` reports whether that happened."""
    n = H.shape[0]
    if n > 12:
        raise ValueError("brute force is limited to n <= 12")
    scale = max(1.0, float(np.max(np.abs(g0))) if n else 1.0)
    gtol = 10.0 * slack * scale
    best = None
    count = 0
    for free_bits in itertools.product((False, True), repeat=n):
        free = np.asarray(free_bits, dtype=bool)
        F = np.nonzero(free)[0]
        Bd = np.nonzero(~free)[0]
        # every lb/ub assignment of the bound spots, one column each
        nb = Bd.size
        ups = np.array(list(itertools.product((0, 1), repeat=nb)), dtype=bool).reshape(2 ** nb, nb).T
        if nb and np.any(ups & ~np.isfinite(ub[Bd])[:, None]):
            keep = ~np.any(ups & ~np.isfinite(ub[Bd])[:, None], axis=0)
            ups = ups[:, keep]
        if ups.shape[1] == 0:
            continue
        K = ups.shape[1]
        X = np.zeros((n, K))
        if nb:
            X[Bd] = np.where(ups, ub[Bd][:, None], lb[Bd][:, None])
        if F.size:
            rhs = g0[F][:, None] - H[np.ix_(F, Bd)] @ X[Bd]
            XF = _chol_solve(H[np.ix_(F, F)], rhs)
            if XF is None:
                continue
            span = np.where(np.isfinite(ub[F]), ub[F] - lb[F], 1.0)
            tol = (slack * np.maximum(1.0, span))[:, None]
            inside = np.all((XF > lb[F][:, None] + tol) & (XF < ub[F][:, None] - tol), axis=0)
            X[F] = XF
        else:
            inside = np.ones(K, dtype=bool)
        G = H @ X - g0[:, None]
        if nb:
            at_lb = ~ups
            ok_b = np.all(np.where(at_lb, G[Bd] >= -gtol, G[Bd] <= gtol), axis=0)
        else:
            ok_b = np.ones(K, dtype=bool)
        good = np.nonzero(inside & ok_b)[0]
        for k in good:
            x = X[:, k]
            f = 0.5 * x @ H @ x - g0 @ x
            lab = np.where(free, 2, np.zeros(n, dtype=int))
            if nb:
                lab[Bd] = ups[:, k].astype(int)
            count += 1
            if best is None or f < best[0]:
                best = (f, x.copy(), lab)
    if best is None:
        raise RuntimeError("no KKT labelling found")
    return best[1], best[2], count == 1


def active_set(W: "wls.Wls", x0: np.ndarray | None = None, tol: float = 1e-12, max_iter: int = 500,
               H=None, g0=None):
    """Projected-Newton polish to a KKT point; returns (x, info)."""
    if H is None or g0 is None:
        H, g0, _ = wls.quadratic_form(W)
    lb, ub = W.lb, W.ub
    n = H.shape[0]
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    x = np.minimum(np.maximum(x, lb), ub)
    scale = max(1.0, float(np.max(np.abs(g0))) if n else 1.0)
    f = lambda v: 0.5 * v @ (H @ v) - g0 @ v
    it = 0
    kkt = np.inf
    for it in range(1, max_iter + 1):
        g = H @ x - g0
        kkt = float(np.max(np.abs(x - np.minimum(np.maximum(x - g, lb), ub)))) / scale if n else 0.0
        if kkt <= tol:
            break
        # variables held at a bound by an outward-pointing gradient (with a small
        # epsilon band so nearly-active variables are also held, as in projected Newton)
        eps = min(1e-8, kkt)
        held = ((x <= lb + eps) & (g > 0)) | ((x >= ub - eps) & (g < 0))
        F = np.nonzero(~held)[0]
        direction = np.zeros(n)
        if F.size:
            step = _chol_solve(H[np.ix_(F, F)], -g[F])
            if step is None:  # semidefinite free block: fall back to a gradient step
                step = -g[F] / max(np.max(np.diag(H)[F]), 1e-300)
            direction[F] = step
        # projected backtracking search along the arc P(x + t d)
        f0 = f(x)
        t = 1.0
        accepted = False
        for _ in range(60):
            xt = np.minimum(np.maximum(x + t * direction, lb), ub)
            if f(xt) <= f0 + 1e-4 * (g @ (xt - x)) or np.array_equal(xt, x):
                accepted = True
                break
            t *= 0.5
        if not accepted or np.array_equal(xt, x):
            # Newton made no progress: one projected gradient step with exact line length
            Hg = H @ g
            gg = g @ g
            a = gg / max(g @ Hg, 1e-300)
            xt = np.minimum(np.maximum(x - a * g, lb), ub)
            if f(xt) > f0:
                break
        x = xt
    return x, dict(iters=it, kkt=kkt)
