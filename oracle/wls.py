"""Objective, gradient, quadratic form and KKT residual (FP64).

Test infrastructure (see the package docstring): never imported by the product.

Notation follows Sec. 2.1: A_s (m x n, one per scenario), row a_{s,i}, weights
w_i >= 0 constant per structure, prescription p, scenario probabilities c_s
(entering through w~_{s,i} = c_s w_i).  All arithmetic is float64; the float32
matrix values of the inputs are widened exactly.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class Wls:
    """FP64 view of one robust WLS problem."""
    A: List[sp.csr_matrix]   # float64 copies of the float32 inputs
    c: np.ndarray            # scenario probabilities c_s
    w: np.ndarray            # per-voxel weights
    p: np.ndarray            # prescription
    lb: np.ndarray
    ub: np.ndarray

    @property
    def m(self) -> int:
        return self.A[0].shape[0]

    @property
    def n(self) -> int:
        return self.A[0].shape[1]

    @property
    def N(self) -> int:
        return len(self.A)


def from_problem(P) -> Wls:
    """Widen a synth.Problem to float64.  A zero probability means 1."""
    A = [sp.csr_matrix((a.val.astype(np.float64), a.col.astype(np.int64), a.row_ptr.astype(np.int64)),
                       shape=(P.m, P.n)) for a in P.A]
    c = np.where(np.asarray(P.prob, dtype=np.float64) == 0.0, 1.0, np.asarray(P.prob, dtype=np.float64))
    w = np.asarray(P.struct_weight, dtype=np.float64)[np.asarray(P.struct_id, dtype=np.int64)]
    return Wls(A=A, c=c, w=w, p=np.asarray(P.presc, dtype=np.float64),
               lb=np.asarray(P.lb, dtype=np.float64), ub=np.asarray(P.ub, dtype=np.float64))


def project(W: Wls, x: np.ndarray) -> np.ndarray:
    """Clip onto the spot-intensity box [lb, ub] (x >= 0 in Sec. 2.1 when lb=0, ub=inf)."""
    return np.minimum(np.maximum(x, W.lb), W.ub)


def scenario_objective(W: Wls, s: int, x: np.ndarray) -> float:
    """f_s(x) = sum_i c_s w_i (a_{s,i}^T x - p_i)^2  (Sec. 2.1, scenario objective;
    c_s is the probability weighting described at the end of Sec. 2.1)."""
    r = W.A[s] @ x - W.p
    return float(W.c[s] * np.sum(W.w * r * r))


def objective(W: Wls, x: np.ndarray) -> float:
    """f(x) = sum_s f_s(x)  (Sec. 2.1, robust problem).  Parity: pinned by the
    quadratic-form identity and by brute force on tiny problems."""
    return float(sum(scenario_objective(W, s, x) for s in range(W.N)))


def scenario_gradient(W: Wls, s: int, x: np.ndarray) -> np.ndarray:
    """grad f_s(x) = sum_i 2 c_s w_i a_{s,i} (a_{s,i}^T x - p_i)  (Sec. 2.1)."""
    r = W.A[s] @ x - W.p
    return 2.0 * W.c[s] * (W.A[s].T @ (W.w * r))


def gradient(W: Wls, x: np.ndarray) -> np.ndarray:
    """grad f(x) = sum_s grad f_s(x).  Parity: pinned by central finite differences."""
    g = np.zeros(W.n)
    for s in range(W.N):
        g += scenario_gradient(W, s, x)
    return g


def scenario_gram(W: Wls, s: int) -> np.ndarray:
    """G_s = A_s^T diag(c_s w) A_s as a dense n x n array (so B_s = G_s + rho/2 I,
    Appendix A, normal equations)."""
    As = W.A[s]
    G = (As.T @ sp.diags(W.c[s] * W.w) @ As).toarray()
    return 0.5 * (G + G.T)


def quadratic_form(W: Wls):
    """(H, g0, const) with f(x) = 1/2 x^T H x - g0^T x + const:
    H = 2 sum_s G_s, g0 = 2 sum_s c_s A_s^T W p, const = sum_s c_s sum_i w_i p_i^2."""
    n = W.n
    H = np.zeros((n, n))
    g0 = np.zeros(n)
    const = 0.0
    for s in range(W.N):
        H += 2.0 * scenario_gram(W, s)
        g0 += 2.0 * W.c[s] * (W.A[s].T @ (W.w * W.p))
        const += W.c[s] * float(np.sum(W.w * W.p * W.p))
    return H, g0, const


def objective_quadratic(H: np.ndarray, g0: np.ndarray, const: float, x: np.ndarray) -> float:
    return float(0.5 * x @ (H @ x) - g0 @ x + const)


def kkt_residual(W: Wls, x: np.ndarray, g0_inf: float | None = None) -> float:
    """Scaled projected-gradient residual ||x - P(x - grad f(x))||_inf / max(1, ||g0||_inf).
    Zero exactly at the minimisers of the box-constrained problem."""
    g = gradient(W, x)
    if g0_inf is None:
        g0 = np.zeros(W.n)
        for s in range(W.N):
            g0 += 2.0 * W.c[s] * (W.A[s].T @ (W.w * W.p))
        g0_inf = float(np.max(np.abs(g0))) if W.n else 0.0
    r = x - project(W, x - g)
    return float(np.max(np.abs(r))) / max(1.0, g0_inf) if W.n else 0.0


def mean_gram_diagonal(W: Wls) -> float:
    """mean_s mean_j (G_s)_jj = mean over scenarios and spots of sum_i c_s w_i a_ij^2.
    Pinned by a hand-worked value and by second differences of f_s."""
    tot = 0.0
    for s in range(W.N):
        As = W.A[s]
        d = np.asarray(As.multiply(As).T @ (W.c[s] * W.w)).ravel()
        tot += float(np.mean(d))
    return tot / W.N


def default_rho(W: Wls, scale: float = 1.0) -> float:
    """Penalty used when the caller gives none (the paper leaves rho to the user,
    Sec. 2.2): rho = 2 * scale * mean diag(G_s), i.e. rho/2 equals the mean
    diagonal of the scenario Gram matrices, which keeps the rule invariant to a
    rescaling of A or w.  Pinned by a hand-worked value and second differences."""
    return 2.0 * scale * mean_gram_diagonal(W)


# --- SpMV references (FP64 products of the float32 inputs) --------------------

def matvec(W: Wls, s: int, v: np.ndarray) -> np.ndarray:
    """A_s v in float64."""
    return W.A[s] @ np.asarray(v, dtype=np.float64)


def matvec_abs(W: Wls, s: int, v: np.ndarray) -> np.ndarray:
    """|A_s| |v|: the scale of each entry of A_s v used by per-entry error bounds."""
    return abs(W.A[s]) @ np.abs(np.asarray(v, dtype=np.float64))


def rmatvec(W: Wls, s: int, t: np.ndarray) -> np.ndarray:
    """A_s^T t in float64."""
    return W.A[s].T @ np.asarray(t, dtype=np.float64)


def rmatvec_abs(W: Wls, s: int, t: np.ndarray) -> np.ndarray:
    """|A_s|^T |t|, the per-entry scale of A_s^T t.  Pinned by a hand-worked value
    and by the triangle inequality (equality for t >= 0)."""
    return abs(W.A[s]).T @ np.abs(np.asarray(t, dtype=np.float64))


def normal_apply(W: Wls, s: int, v: np.ndarray, rho: float) -> np.ndarray:
    """B_s v = (A_s^T diag(c_s w) A_s + rho/2 I) v  (Appendix A).  Pinned by a
    hand-worked value and by the gradient identity
    B_s v = (grad f_s(v) - grad f_s(0)) / 2 + rho/2 v."""
    v = np.asarray(v, dtype=np.float64)
    return W.A[s].T @ (W.c[s] * W.w * (W.A[s] @ v)) + 0.5 * rho * v


def normal_apply_abs(W: Wls, s: int, v: np.ndarray, rho: float) -> np.ndarray:
    """(|A_s|^T diag(c_s w) |A_s| + rho/2 I) |v|, the per-entry scale of B_s v.
    Pinned by a hand-worked value and by the triangle inequality."""
    av = np.abs(np.asarray(v, dtype=np.float64))
    aA = abs(W.A[s])
    return aA.T @ (W.c[s] * W.w * (aA @ av)) + 0.5 * rho * av
