"""Edge cases of the GPU path against closed forms and the oracle's minimiser:
a single spot (the minimiser has a closed form), a spot count one past a
64-column tile (a tile holding one column), and degenerate inputs (empty
voxel rows, a structure of weight zero, a scenario with no nonzeros)."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

import synth
from oracle import exact, wls

pytestmark = pytest.mark.gpu


def _exact(P):
    W = wls.from_problem(P)
    Hm, g0, _ = wls.quadratic_form(W)
    xs, _ = exact.active_set(W, H=Hm, g0=g0)
    return W, xs, wls.objective(W, xs)


@pytest.mark.parametrize("xupdate", ["dense", "cg"])
def test_single_spot_reaches_the_closed_form_minimiser(xupdate):
    """With one spot, f(x) = q x^2 - 2 r x + const, so x* = clip(r / q, lb, ub)."""
    import paper_2304_14568_amd as A
    P = synth.make_tiny(4, spots=(1, 1), num_scen=3, probs=[0.5, 0.3, 0.2])
    W = wls.from_problem(P)
    q = sum(W.c[s] * float(np.sum(W.w * (W.A[s] @ np.ones(1)) ** 2)) for s in range(W.N))
    r = sum(W.c[s] * float(np.sum(W.w * (W.A[s] @ np.ones(1)) * W.p)) for s in range(W.N))
    xstar = float(np.clip(r / q, W.lb[0], W.ub[0]))
    assert 0 < xstar < W.ub[0]
    with A.Solver(P, xupdate=xupdate, max_iter=3000) as S:
        zs, info, st = S.solve()
        assert st == 0, info
        assert abs(zs[0][0] - xstar) <= 1e-5 * xstar
        x, pinfo, pst = S.pgd(0, obj_rel_tol=1e-12, max_iter=2000)
        assert abs(x[0] - xstar) <= 1e-5 * xstar


@pytest.mark.parametrize("xupdate", ["dense", "cg"])
def test_one_column_past_a_tile(xupdate):
    """65 spots: the dense path's second 64-block holds a single column."""
    import paper_2304_14568_amd as A
    P = synth.make_tiny(5, spots=(5, 13), num_scen=3)
    assert P.n == 65
    W, xs, fs = _exact(P)
    with A.Solver(P, xupdate=xupdate, max_iter=4000) as S:
        zs, info, st = S.solve()
        assert st == 0, info
        assert abs(wls.objective(W, zs[0]) - fs) <= 1e-5 * fs
        if xupdate == "dense":
            x, pinfo, _ = S.pgd(0, obj_rel_tol=1e-12, max_iter=20000)
            assert abs(wls.objective(W, x) - fs) <= 1e-6 * fs


def _degenerate():
    """Empty voxel rows in one scenario, a zero-weight structure, and an extra
    scenario without any nonzero."""
    P = synth.make_tiny(6, num_scen=3)
    a = P.A[0]
    rows = np.diff(a.row_ptr)
    keep = np.ones(P.m, dtype=bool)
    keep[: P.m // 4] = False                      # the first quarter of the voxels: no dose in scenario 0
    nz_keep = np.repeat(keep, rows)
    new_rows = np.where(keep, rows, 0)
    A0 = synth.Csr(row_ptr=np.concatenate([[0], np.cumsum(new_rows)]).astype(np.int64),
                   col=a.col[nz_keep].copy(), val=a.val[nz_keep].copy())
    empty = synth.Csr(row_ptr=np.zeros(P.m + 1, dtype=np.int64), col=np.zeros(0, dtype=np.int32),
                      val=np.zeros(0, dtype=np.float32))
    sw = P.struct_weight.copy()
    assert sw.shape[0] == 3 and sw[1] > sw[2] > 0  # normal tissue, target, organ at risk
    sw[2] = 0.0                                   # the organ at risk weighs nothing
    return dataclasses.replace(P, A=[A0, P.A[1], P.A[2], empty], prob=np.array([0.4, 0.3, 0.2, 0.1]),
                               struct_weight=sw)


@pytest.mark.parametrize("xupdate", ["dense", "cg"])
def test_degenerate_inputs(xupdate):
    import paper_2304_14568_amd as A
    P = _degenerate()
    W, xs, fs = _exact(P)
    with A.Solver(P, xupdate=xupdate, max_iter=4000) as S:
        zs, info, st = S.solve()
        assert st == 0, info
        assert abs(wls.objective(W, zs[0]) - fs) <= 1e-5 * fs
        # the objective and products of the empty scenario are exact zeros / the prescription term
        rng = np.random.default_rng(1)
        v = rng.uniform(0, 1, P.n).astype(np.float32)
        assert np.all(S.matvec(v, 3) == 0.0)
        assert abs(S.objective(zs[0]) - wls.objective(W, zs[0])) <= 1e-6 * fs
