"""The device-driven PGD on the packed fp64 sum of the Gram matrices against
the FP64 oracle PGD (Sec. 2.1).  Both run the same backtracking rule on the same
quadratic (fp32-exact matrix values, fp64 arithmetic), so they take the same
steps: the iterates agree to rounding, not only the final objective."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import exact, pgd as opgd, wls

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def probs():
    out = []
    for P in (synth.make_tiny(2), synth.hn_small(6)):
        W = wls.from_problem(P)
        Hm, g0, _ = wls.quadratic_form(W)
        xs, _ = exact.active_set(W, H=Hm, g0=g0)
        out.append((P, W, xs, wls.objective(W, xs)))
    return out


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("iters", [1, 7, 40])
def test_dense_pgd_iterates_follow_the_oracle(probs, which, iters):
    import paper_2304_14568_amd as A
    P, W, xs, fs = probs[which]
    q = opgd.pgd_armijo(W, obj_rel_tol=0.0, max_iter=iters, record=False)
    with A.Solver(P, xupdate="dense") as S:
        x, info, st = S.pgd(0, obj_rel_tol=0.0, max_iter=iters, dense=1)
    assert st == A.MAX_ITER
    assert info["iter"] == q.iters
    assert abs(info["tau"] - q.alpha) <= 1e-10 * q.alpha          # power iteration on the same H
    assert np.linalg.norm(x - q.x) <= 1e-9 * np.linalg.norm(q.x)
    assert abs(info["obj"] - q.obj) <= 1e-11 * q.obj
    assert abs(info["obj"] - wls.objective(W, x)) <= 1e-11 * q.obj


@pytest.mark.parametrize("which", [0, 1])
def test_dense_pgd_stops_where_the_oracle_stops(probs, which):
    import paper_2304_14568_amd as A
    P, W, xs, fs = probs[which]
    q = opgd.pgd_armijo(W, record=False)           # relative objective change 1e-5
    with A.Solver(P, xupdate="dense") as S:
        x, info, st = S.pgd(0)                     # dense form chosen by default here
    assert q.converged and st == 0
    assert info["iter"] == q.iters
    assert abs(info["obj"] - q.obj) <= 1e-10 * q.obj
    assert info["obj"] >= fs * (1 - 1e-12)


def test_dense_pgd_reaches_the_minimum(probs):
    import paper_2304_14568_amd as A
    P, W, xs, fs = probs[0]
    with A.Solver(P, xupdate="dense") as S:
        x, info, st = S.pgd(0, obj_rel_tol=1e-12, max_iter=20000)
        # the sparse form (fp32 iterates) agrees on the minimum within its precision
        xsp, info_sp, _ = S.pgd(0, obj_rel_tol=1e-9, max_iter=5000, dense=0)
    f = wls.objective(W, x)
    assert f >= fs * (1 - 1e-12)
    assert abs(f - fs) <= 1e-7 * fs, (f, fs)
    assert abs(wls.objective(W, xsp) - fs) <= 1e-4 * fs


def test_dense_pgd_backtracking_limits(probs):
    """A first step far too long for the trial budget fails the line search
    (status MAX_ITER after no accepted step); a budget that reaches a good step
    in a later round of trial points accepts it as the sequential search would."""
    import paper_2304_14568_amd as A
    P, W, xs, fs = probs[1]
    alpha0 = 10.0 / opgd.lipschitz(W)
    big = alpha0 * 2.0 ** 20
    with A.Solver(P, xupdate="dense") as S:
        x, info, st = S.pgd(0, alpha=big, max_trials=5, max_iter=3)
        assert st == A.MAX_ITER and info["iter"] == 0
        x, info, st = S.pgd(0, alpha=big, max_trials=60, max_iter=3, obj_rel_tol=0.0)
    q = opgd.pgd_armijo(W, alpha=big, max_trials=60, max_iter=3, obj_rel_tol=0.0, record=False)
    assert info["iter"] == q.iters == 3
    assert np.linalg.norm(x - q.x) <= 1e-9 * np.linalg.norm(q.x)


def test_dense_pgd_needs_the_dense_context(probs):
    import paper_2304_14568_amd as A
    P = probs[0][0]
    with A.Solver(P, xupdate="cg") as S:
        with pytest.raises(A.AdmmError):
            S.pgd(0, dense=1)
        with pytest.raises(A.AdmmError):
            S.pgd(0, dense=2)                      # not -1, 0 or 1
        x, info, st = S.pgd(0)                     # default falls back to the sparse form
        assert info["iter"] > 0


def test_dense_pgd_from_a_start_point_and_in_a_batch(probs):
    import paper_2304_14568_amd as A
    (P0, W0, _, _), (P1, W1, _, _) = probs
    x0 = np.linspace(-1.0, 3.0, P1.n)
    q = opgd.pgd_armijo(W1, x0=x0, obj_rel_tol=0.0, max_iter=10, record=False)
    with A.Solver([P0, P1], xupdate="dense") as S:
        x, info, st = S.pgd(1, x0=x0, obj_rel_tol=0.0, max_iter=10)
    assert np.linalg.norm(x - q.x) <= 1e-9 * np.linalg.norm(q.x)


def test_stream_probe_reports_a_plausible_rate():
    import paper_2304_14568_amd as A
    gbs = A.stream_probe(64 << 20, reps=5)
    assert 100.0 < gbs < 20000.0, gbs
