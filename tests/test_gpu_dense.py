"""The dense x-update (cached inverse of every A_s^T c_s W A_s + rho/2 I, the
exact subproblem solve of Appendix A) against the FP64 oracle, whose ADMM-BB
also solves every subproblem exactly (Cholesky): the iterates themselves must
agree, not only the final objective."""
from __future__ import annotations

import dataclasses

import numpy as np
import pytest

import synth
from oracle import admm as oadmm, exact, wls

pytestmark = pytest.mark.gpu


def _oracle_path(W, iters, rho=None, z0=None, z_mode=0):
    zs, fs = [], []
    oadmm.admm_bb(W, rho=rho, max_iter=iters, obj_rel_tol=0.0, eps_abs=0.0, eps_rel=0.0, z0=z0, record=False,
                  z_mode=z_mode, callback=lambda k, z, f: (zs.append(z.copy()), fs.append(f)))
    return zs, fs


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
def test_dense_iterates_follow_the_oracle(probs, which):
    """z after k iterations, and every scalar of the first K iterations (the
    objective, the Barzilai-Borwein step tau, both residuals and both
    tolerances of Sec. 2.2), against the oracle's history.  The device keeps
    the inverses in fp32 and the iterates in fp32; over the first ten
    iterations it was measured within 1.4e-5 (tau), 2.7e-6 (r_prim), 7.3e-7
    (r_dual) and 2.1e-8 (objective) of the oracle; the bounds leave 4-8x."""
    import paper_2304_14568_amd as A
    P, W, xs, fs = probs[which]
    K = 12
    zr, fr = _oracle_path(W, K)
    # the paper's tolerances: the stopping test is evaluated, and does not
    # pass, within K iterations
    hist = oadmm.admm_bb(W, max_iter=K, record=True).history
    assert len(hist) == K
    with A.Solver(P, xupdate="dense", max_iter=1000) as S:
        assert S.xupdate()[0] == "dense"
        assert abs(S.rho() - wls.default_rho(W)) <= 1e-6 * S.rho()
        for k in (1, 2, 3, 6, K):
            S.reset()
            S.iterate(k)
            z = S.z()
            # fp32 inverse and fp32 iterates against fp64 Cholesky solves
            err = np.linalg.norm(z - zr[k - 1]) / max(1e-30, np.linalg.norm(zr[k - 1]))
            assert err <= 2e-5 * k, (k, err)
        tr = S.trace()
        assert len(tr) >= K
        for t in tr[:K]:
            k = t["iter"]
            h = hist[k - 1]
            assert abs(t["obj"] - fr[k - 1]) <= 1e-7 * fr[k - 1]
            for key, tol in (("obj", 1e-7), ("tau", 1e-4), ("r_prim", 2e-5), ("r_dual", 2e-5),
                             ("eps_prim", 2e-5), ("eps_dual", 1e-4)):
                assert abs(t[key] - h[key]) <= tol * abs(h[key]), (k, key, t[key], h[key])
        # the objective from the quadratic form (fp64 Gram matrix, fp64 p) equals the
        # sparse-pass objective at the same z up to the fp32 rounding of p in the pass
        assert abs(tr[K - 1]["obj"] - S.objective(S.z())) <= 1e-7 * tr[K - 1]["obj"]
        assert abs(tr[K - 1]["obj"] - wls.objective(W, S.z())) <= 1e-9 * tr[K - 1]["obj"]


@pytest.mark.parametrize("z_mode,spots,num_scen", [(0, (9, 11), 20), (1, (9, 11), 20), (0, (3, 4), 2),
                                                   (0, (8, 8), 5)])
def test_dense_iterates_with_more_scenarios_than_waves(z_mode, spots, num_scen):
    """x_s and the z-update are formed with one wave per scenario at a time,
    sixteen waves per workgroup: with 20 scenarios four waves take a second
    scenario, whose x_s, dual and residual terms enter the fixed-order sums
    after their first.  9 x 11 = 99 spots: the last 16-spot group of the last
    64-spot block holds 3 spots.  z after k iterations and the objective
    trace against the oracle, at the bounds of the 13-scenario test, for both
    z-updates (the projected average of x_s + y_s / rho, and the literal
    reading that averages x_s alone).  Also 12 spots (three of the four
    workgroups of the only block hold none) and exactly 64 (no ragged
    block)."""
    import paper_2304_14568_amd as A
    P = synth.make_tiny(4, spots=spots, num_scen=num_scen,
                        range_scales=tuple(np.linspace(0.96, 1.04, num_scen)))
    assert P.num_scen == num_scen and P.n == spots[0] * spots[1]
    W = wls.from_problem(P)
    K = 8
    zr, fr = _oracle_path(W, K, z_mode=z_mode)
    # the paper's stopping test does not pass within K iterations
    assert len(oadmm.admm_bb(W, max_iter=K, record=True, z_mode=z_mode).history) == K
    Hm, g0, _ = wls.quadratic_form(W)
    lmax = float(np.linalg.eigvalsh(Hm)[-1])
    with A.Solver(P, xupdate="dense", max_iter=1000, z_mode=z_mode) as S:
        assert S.xupdate()[0] == "dense"
        for k in (1, 2, 5, K):
            S.reset()
            S.iterate(k)
            z = np.asarray(S.z(), dtype=np.float64)
            err = np.linalg.norm(z - zr[k - 1]) / max(1e-30, np.linalg.norm(zr[k - 1]))
            assert err <= 2e-5 * k, (k, err)
            t = S.trace()[-1]
            assert t["iter"] == k
            # the device's objective is f at its own iterate (48-bit sum of the
            # Gram matrices, fp64 sums) ...
            fz = wls.objective(W, z)
            assert abs(t["obj"] - fz) <= 1e-9 * fz, (k, t["obj"], fz)
            # ... so it differs from the oracle's by what the iterates' difference
            # dz moves the quadratic f = z'Hz/2 - g0'z + c: at most
            # |grad f| |dz| + lmax(H) |dz|^2 / 2 (tiny problems with few spots
            # have large gradients next to f: the 12-spot case measured 1.6e-7
            # relative at k = 7)
            dz = np.linalg.norm(z - zr[k - 1])
            grad = Hm @ zr[k - 1] - g0
            bound = np.linalg.norm(grad) * dz + 0.5 * lmax * dz * dz + 1e-9 * fr[k - 1]
            assert abs(t["obj"] - fr[k - 1]) <= bound, (k, t["obj"], fr[k - 1], bound)


@pytest.mark.parametrize("which", [0, 1])
def test_dense_solve_reaches_the_minimum(probs, which):
    import paper_2304_14568_amd as A
    P, W, xs, fs = probs[which]
    with A.Solver(P, xupdate="dense", max_iter=3000) as S:
        zs, info, st = S.solve()
        assert st == 0, info
        f = wls.objective(W, zs[0])
        assert abs(f - fs) <= 1e-5 * fs, (f, fs)
        assert info[0]["cg_steps"] == 0


def test_dense_penalty_change_refactors(probs):
    """A new rho rebuilds the cached inverses: the iterates then follow the
    oracle run at that rho."""
    import paper_2304_14568_amd as A
    P, W, xs, fs = probs[1]
    rho2 = 3.0 * wls.default_rho(W)
    zr, _ = _oracle_path(W, 5, rho=rho2)
    with A.Solver(P, xupdate="dense") as S:
        S.iterate(4)
        S.warm_start(0, None, rho2)
        S.iterate(5)
        z = S.z()
        assert np.linalg.norm(z - zr[4]) / np.linalg.norm(zr[4]) <= 1e-3


def test_dense_batch_and_cg_agree_on_the_minimum(probs):
    import paper_2304_14568_amd as A
    Ps = [probs[0][0], probs[1][0]]
    with A.Solver(Ps, xupdate="dense", max_iter=3000) as S:
        zs, infos, st = S.solve()
    for (P, W, xs, fs), z in zip(probs, zs):
        assert abs(wls.objective(W, z) - fs) <= 1e-5 * fs


def test_auto_selects_dense_for_small_problems(probs):
    """The form is chosen before packing: the dense form gets the chunk-row
    layout alone under the automatic layout choice, the sliced one only when
    asked for (its passes then agree with the chunk-row ones)."""
    import paper_2304_14568_amd as A
    P, W = probs[1][0], probs[1][1]
    with A.Solver(P, xupdate="auto") as S:
        assert S.xupdate()[0] == "dense"
        assert S.tuning()["format"] == "csr"
        v = np.linspace(0.1, 1.0, P.n).astype(np.float32)
        q_csr = S.normal_apply(v, 1)
        rho = S.rho()
    with A.Solver(P, xupdate="auto", format="sell") as S:
        assert S.xupdate()[0] == "dense"
        assert S.tuning()["format"] == "sell"
        q_sell = S.normal_apply(v, 1)
    ref = wls.normal_apply(W, 1, v, rho)
    scale = wls.normal_apply_abs(W, 1, v, rho)
    assert np.all(np.abs(q_csr - ref) <= 1e-6 * scale)
    assert np.all(np.abs(q_sell - ref) <= 1e-6 * scale)
    with A.Solver(probs[0][0], xupdate="cg") as S:
        assert S.xupdate()[0] == "cg"


def test_dense_checkpoint_resume_is_exact(probs):
    import paper_2304_14568_amd as A
    P = probs[1][0]
    with A.Solver(P, xupdate="dense", use_graph=0) as S:
        S.iterate(5)
        saved = S.get_state()
        S.iterate(6)
        za = S.z()
        S.set_state(saved)
        S.iterate(6)
        assert np.array_equal(S.z(), za)


def test_dense_setup_in_scenario_chunks_matches_one_chunk(probs, monkeypatch):
    """The cached inverses built one scenario at a time (the memory-bounded
    set-up) give the same iterates as the set-up of all scenarios at once."""
    import paper_2304_14568_amd as A
    P = probs[1][0]
    with A.Solver(P, xupdate="dense", use_graph=0) as S:
        S.iterate(15)
        z_one = S.z()
    monkeypatch.setenv("ADMMBB_DENSE_CHUNK_MB", "1")  # below one scenario: chunks of 1
    with A.Solver(P, xupdate="dense", use_graph=0) as S:
        S.iterate(15)
        z_chunked = S.z()
    # the Gram matrices sum with fp64 atomics (order-dependent in the last bits)
    assert np.linalg.norm(z_chunked - z_one) <= 1e-6 * np.linalg.norm(z_one)


def test_dense_x_update_near_its_size_limit():
    """n = 7 895 spots (124 blocks of 64, the limit is 127): the first x-update
    from z = 0, y = 0 solves B_s x_s = b_s (checked with the fp64 operator of
    the oracle, to the fp32 rounding of the cached inverse amplified by the
    conditioning of B_s), and the dense and CG x-updates reach the same
    objective."""
    import paper_2304_14568_amd as A
    P = synth.make_hn(seed=7, grid=(72, 72, 48), body_semi_vox=(30, 24, 18), target_size=1.1, num_layers=11,
                      spot_spacing=2.5, num_scen=2)
    assert 7800 < P.n <= 8128
    W = wls.from_problem(P)
    with A.Solver(P, xupdate="dense", max_iter=3000) as S:
        rho = S.rho()
        S.iterate(1)
        st = S.get_state()
        z = st["z"]
        d = np.asarray(st["d"]).reshape(P.num_scen, P.n)
        for s in range(P.num_scen):
            x = d[s] + z
            b = W.A[s].T @ (W.c[s] * W.w * W.p)
            r = wls.normal_apply(W, s, x, rho) - b
            assert np.linalg.norm(r) <= 2e-4 * np.linalg.norm(b), np.linalg.norm(r) / np.linalg.norm(b)
        S.reset()
        zs, info, stt = S.solve()
        assert stt == 0, info
        f_dense = wls.objective(W, zs[0])
    with A.Solver(P, xupdate="cg", max_iter=3000) as S:
        zc, infoc, stc = S.solve()
        assert stc == 0, infoc
        f_cg = wls.objective(W, zc[0])
    assert abs(f_dense - f_cg) <= 1e-5 * f_cg, (f_dense, f_cg)


def _long_segment_problem():
    """n = 130 spots (64-column blocks of 64, 64 and 2 columns) with three rows
    planted in scenario 0: columns {0} and 64..127 (65 nonzeros; the stored row
    is padded to a multiple of 4 by repeating column 127, so block 1 holds 67
    entries), every column (130) and columns 0..127 (128, no padding).  Their
    values exceed every other entry, so a lost or doubled product shows."""
    P = synth.make_tiny(3, spots=(10, 13), num_scen=2)
    assert P.n == 130
    a = P.A[0]
    rng = np.random.default_rng(11)
    rows = [(a.col[a.row_ptr[i]:a.row_ptr[i + 1]], a.val[a.row_ptr[i]:a.row_ptr[i + 1]]) for i in range(P.m)]
    planted = [np.concatenate([[0], np.arange(64, 128)]), np.arange(130), np.arange(128)]
    vmax = float(a.val.max())
    for r, cols in zip(np.flatnonzero(P.struct_id == 1)[:3], planted):
        rows[r] = (cols.astype(np.int32), (vmax * rng.uniform(1.0, 2.0, cols.size)).astype(np.float32))
    lens = np.array([c.size for c, _ in rows])
    A0 = synth.Csr(row_ptr=np.concatenate([[0], np.cumsum(lens)]).astype(np.int64),
                   col=np.concatenate([c for c, _ in rows]).astype(np.int32),
                   val=np.concatenate([v for _, v in rows]).astype(np.float32))
    return dataclasses.replace(P, A=[A0, P.A[1]])


def _first_x_update(P, monkeypatch, atomic):
    """x_s after one iteration from z = 0, y = 0 (the solutions of B_s x_s = b_s),
    with the Gram matrices formed by per-tile lists or by global atomics."""
    import paper_2304_14568_amd as A
    if atomic:
        monkeypatch.setenv("ADMMBB_GRAM_ATOMIC", "1")
    else:
        monkeypatch.delenv("ADMMBB_GRAM_ATOMIC", raising=False)
    with A.Solver(P, xupdate="dense") as S:
        assert S.xupdate()[0] == "dense"
        rho = S.rho()
        S.iterate(1)
        st = S.get_state()
    monkeypatch.delenv("ADMMBB_GRAM_ATOMIC", raising=False)
    z = np.asarray(st["z"])
    d = np.asarray(st["d"]).reshape(P.num_scen, P.n)
    return rho, d + z[None, :]


@pytest.mark.parametrize("which", ["planted", "hn_small"])
def test_tile_gram_matches_the_normal_equations_and_the_atomic_gram(which, monkeypatch):
    P = _long_segment_problem() if which == "planted" else synth.hn_small(6)
    W = wls.from_problem(P)
    rho, x_tile = _first_x_update(P, monkeypatch, atomic=False)
    rho_a, x_atom = _first_x_update(P, monkeypatch, atomic=True)
    assert rho == rho_a
    for s in range(P.num_scen):
        b = W.A[s].T @ (W.c[s] * W.w * W.p)
        r = wls.normal_apply(W, s, x_tile[s], rho) - b
        assert np.linalg.norm(r) <= 1e-4 * np.linalg.norm(b), np.linalg.norm(r) / np.linalg.norm(b)
        # both Gram paths give the same inverse up to its fp32 rounding
        assert np.linalg.norm(x_tile[s] - x_atom[s]) <= 1e-6 * np.linalg.norm(x_atom[s])


def test_dense_set_up_and_iterations_are_bitwise_reproducible(monkeypatch):
    """The Gram tiles are summed in 64-bit fixed point (exact, independent of
    the order of the atomics) and everything after them in fixed order, so two
    contexts of the same problem produce identical iterates."""
    import paper_2304_14568_amd as A
    monkeypatch.delenv("ADMMBB_GRAM_ATOMIC", raising=False)
    P = synth.hn_small(6)
    states = []
    for _ in range(2):
        with A.Solver(P, xupdate="dense") as S:
            S.iterate(5)
            st = S.get_state()
            states.append((np.asarray(st["z"]).copy(), np.asarray(st["y"]).copy(), np.asarray(st["d"]).copy(),
                           S.objective(st["z"])))
    (z0, y0, d0, f0), (z1, y1, d1, f1) = states
    assert np.array_equal(z0, z1) and np.array_equal(y0, y1) and np.array_equal(d0, d1)
    assert f0 == f1


def _run_both_orders(Ps, **kw):
    import paper_2304_14568_amd as A
    out = {}
    for nl in (4, 3):
        with A.Solver(Ps, xupdate="dense", dense_launches=nl, max_iter=3000, **kw) as S:
            S.iterate(7)
            st7 = [S.get_state(p) for p in range(len(Ps))]
            S.reset()
            zs, info, status = S.solve()
            out[nl] = (st7, zs, info, [S.trace(p) for p in range(len(Ps))], status)
    return out[4], out[3]


@pytest.mark.parametrize("case", ["tiny", "hn_small", "batch_of_both", "no_graph"])
def test_three_launch_iteration_equals_four_launch_order(probs, case):
    """The three-launch dense iteration (the stopping test of an iteration
    beside the next x-update, the dual update beside the Barzilai-Borwein step
    that every wave forms itself) against the four-launch order: the same
    duals, differences and scalars after 7 iterations, and the same solve
    (iterates, trace and stopping decision of every patient), bit for bit.
    The batch stops its two patients at different iterations."""
    Ps = {"tiny": [probs[0][0]], "hn_small": [probs[1][0]], "batch_of_both": [probs[0][0], probs[1][0]],
          "no_graph": [probs[1][0]]}[case]
    a, b = _run_both_orders(Ps, **({"use_graph": 0} if case == "no_graph" else {}))
    for sa, sb in zip(a[0], b[0]):
        for key in ("z", "y", "d", "scalars"):
            assert np.array_equal(sa[key], sb[key]), key
    for za, zb in zip(a[1], b[1]):
        assert np.array_equal(za, zb)
    assert a[2] == b[2]
    assert a[3] == b[3]
    assert a[4] == b[4]
    if case == "batch_of_both":
        assert a[2][0]["iter"] != a[2][1]["iter"]
