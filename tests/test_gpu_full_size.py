"""GPU parity at the full head-and-neck size (about 250k voxels, 2 981 spots,
13 scenarios, 8e7 nonzeros): the workload and launch configuration that
`bench.py` times, against FP64 definitions and the oracle's stored minimum.

  * every entry of A_s v, A_s^T t and B_s v for three scenarios against the
    fp64 product of the same fp32 inputs (per entry <= 1e-6 (|A||v|)_i);
  * f and grad f at a point against the fp64 definitions;
  * the default solve (dense x-update, the paper's stopping rule) against the
    oracle's active-set minimiser stored in tests/golden (objective 1e-5, KKT
    residual 1e-6);
  * spot intensities within 1e-4 in l2 at the solver's own stop with residual
    tolerances 1e-7, for the dense x-update and the CG x-update in fp32, bf16
    and fp16 (KKT residual asserted, kappa(H) printed);
  * the CG forms at the paper's stop against the same minimum;
  * the dense PGD with its relative-change stop against the same minimum.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import wls
from tests.golden.refs import load

pytestmark = pytest.mark.gpu

SPMV_TOL = 1e-6


@pytest.fixture(scope="module")
def full():
    P = synth.hn_full(0)
    rec, xs = load("hn_full_s0")
    assert rec is not None and rec["digest"] == P.digest(), "stored oracle minimum missing or stale"
    W = wls.from_problem(P)
    print(f"[full] m={P.m} n={P.n} N={P.num_scen} nnz={P.nnz} kappa(H)={rec['cond_H']:.3g}", flush=True)
    return P, W, rec["f_star"], xs, rec["cond_H"]


def _per_entry(got, ref, scale):
    err = np.abs(np.asarray(got, dtype=np.float64) - ref)
    bound = SPMV_TOL * scale + 1e-30
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, f"{bad.size} entries over bound; worst ratio {np.max(err / bound):.3g}"


@pytest.mark.parametrize("fmt", ["csr", "sell"])
def test_full_size_products(full, fmt):
    import paper_2304_14568_amd as A
    P, W, _, _, _ = full
    rng = np.random.default_rng(21)
    with A.Solver(P, format=fmt) as S:
        rho = S.rho()
        for s in (0, 6, P.num_scen - 1):
            v = rng.uniform(0, 1, P.n).astype(np.float32)
            _per_entry(S.matvec(v, s), wls.matvec(W, s, v), wls.matvec_abs(W, s, v))
            t = rng.normal(size=P.m).astype(np.float32)
            _per_entry(S.rmatvec(t, s), wls.rmatvec(W, s, t), wls.rmatvec_abs(W, s, t))
            _per_entry(S.normal_apply(v, s), wls.normal_apply(W, s, v, rho), wls.normal_apply_abs(W, s, v, rho))


def test_full_size_objective_and_gradient(full):
    import paper_2304_14568_amd as A
    P, W, fs, xs, _ = full
    rng = np.random.default_rng(22)
    x = (xs * rng.uniform(0.5, 1.5, P.n)).astype(np.float32).astype(np.float64)
    with A.Solver(P) as S:
        f = S.objective(x)
        g, f2 = S.gradient(x)
    f_ref = wls.objective(W, x)
    g_ref = wls.gradient(W, x)
    # the sparse pass reads p in fp32: the objective carries its rounding
    assert abs(f - f_ref) <= 1e-6 * f_ref
    assert abs(f2 - f_ref) <= 1e-6 * f_ref
    scale = np.zeros(P.n)
    for s in range(W.N):
        r_abs = abs(W.A[s]) @ x + W.p
        scale += 2 * W.c[s] * (abs(W.A[s]).T @ (W.w * r_abs))
    _per_entry(g, g_ref, scale)


def _intensity_err(z, xs):
    return float(np.linalg.norm(z - xs) / np.linalg.norm(xs))


def test_full_size_default_solve_matches_the_oracle_minimum(full):
    """The configuration bench.py times, stopped by the paper's rule (Sec. 2.2
    residual tolerances 1e-6 and Sec. 2.3 objective change): objective within
    1e-5 of f*, KKT residual <= 1e-6 (reported by admm_solve, checked against
    the fp64 definition).  At these tolerances the intensities are identified
    to about 1.4e-4 only: kappa(H) = 2.7e4 on this workload."""
    import paper_2304_14568_amd as A
    P, W, fs, xs, cond = full
    with A.Solver(P, max_iter=3000) as S:
        assert S.xupdate()[0] == "dense"
        zs, info, st = S.solve()
        assert st == 0, info
        z = zs[0]
        kkt = wls.kkt_residual(W, z)
        err = _intensity_err(z, xs)
        print(f"[full] kappa(H) {cond:.3g}; paper stop: {info[0]['iter']} it, gap "
              f"{(wls.objective(W, z) - fs) / fs:.2e}, kkt {kkt:.2e} (library {info[0]['kkt']:.2e}), "
              f"z err {err:.2e}", flush=True)
        assert abs(wls.objective(W, z) - fs) <= 1e-5 * fs
        assert abs(info[0]["obj"] - wls.objective(W, z)) <= 1e-9 * fs
        assert kkt <= 1e-6 and info[0]["kkt"] <= 1e-6
        assert abs(info[0]["kkt"] - kkt) <= 0.2 * kkt + 1e-8
        assert err <= 2e-4, err


@pytest.mark.parametrize("xupdate,precision", [("dense", "fp32"), ("cg", "fp32"), ("cg", "bf16"), ("cg", "fp16")])
def test_full_size_intensities_at_the_tight_stop(full, xupdate, precision):
    """Spot intensities within 1e-4 (l2, relative) of the oracle's x* once the
    run has converged: residual tolerances eps_abs = eps_rel = 1e-7, which the
    solver's own stopping rule meets at a KKT residual near 1e-7 (asserted
    <= 1e-6) for the dense x-update and for the CG x-update with fp32, bf16 and
    fp16 values (the reduced-precision forms keep the fp32 residual as their
    outer correction)."""
    import paper_2304_14568_amd as A
    P, W, fs, xs, cond = full
    with A.Solver(P, max_iter=3000, xupdate=xupdate, precision=precision, eps_abs=1e-7, eps_rel=1e-7) as S:
        zs, info, st = S.solve()
        assert st == 0, info
        z = zs[0]
        f = wls.objective(W, z)
        kkt = wls.kkt_residual(W, z)
        err = _intensity_err(z, xs)
        print(f"[full] {xupdate} {precision} kappa(H) {cond:.3g}: {info[0]['iter']} it, gap {(f - fs) / fs:.2e}, "
              f"kkt {kkt:.2e}, z err {err:.2e}", flush=True)
        assert abs(f - fs) <= 1e-5 * fs
        assert kkt <= 1e-6 and info[0]["kkt"] <= 1e-6
        assert err <= 1e-4, err


@pytest.mark.parametrize("precision", ["fp32", "bf16", "fp16"])
def test_full_size_cg_forms_match_the_oracle_minimum(full, precision):
    import paper_2304_14568_amd as A
    P, W, fs, xs, cond = full
    with A.Solver(P, max_iter=3000, xupdate="cg", precision=precision) as S:
        zs, info, st = S.solve()
        assert st == 0, info
        f = wls.objective(W, zs[0])
        print(f"[full] cg {precision}: {info[0]['iter']} it, gap {(f - fs) / fs:.2e}, "
              f"z err {_intensity_err(zs[0], xs):.2e}", flush=True)
        assert abs(f - fs) <= 1e-5 * fs
        assert info[0]["kkt"] <= 1e-6


def test_full_size_dense_pgd_matches_the_oracle_minimum(full):
    """PGD with the paper's relative-change stop (Sec. 2.1, here at 1e-11)
    against the oracle's f*.  The Gram sums behind the dense PGD are exact
    (fixed point), so the set-up and every PGD iterate are the same in every
    run: two runs stop at the same iteration with the same point."""
    import paper_2304_14568_amd as A
    P, W, fs, xs, cond = full
    runs = []
    for _ in range(2):
        with A.Solver(P) as S:
            runs.append(S.pgd(0, obj_rel_tol=1e-11, max_iter=5000))
    (x, info, st), (x2, info2, st2) = runs
    f = wls.objective(W, x)
    print(f"[full] dense pgd: {info['iter']} it, status {st}, gap {(f - fs) / fs:.2e}", flush=True)
    assert st == 0 and st2 == 0
    assert info["iter"] == info2["iter"] and np.array_equal(x, x2)
    assert f >= fs * (1 - 1e-9)
    assert abs(f - fs) <= 1e-5 * fs
    assert abs(info["obj"] - f) <= 1e-9 * fs
