"""GPU parity of the HIP path against the FP64 oracle (through the C-ABI).

Tolerances:
  SpMV-type products (fp32 values, fp32/fp64 accumulation): per entry
      |y_gpu - y_ref| <= 1e-6 * (|A| |v|)_i      (y_ref = fp64 product of the same fp32 inputs)
  final objective: |f_gpu - f*| <= 1e-5 f*
  spot intensities: ||z - x*|| / ||x*|| <= 1e-4 once converged: at the
      solver's own stop with residual tolerances 1e-7, with the KKT residual
      asserted <= 1e-6 and kappa(H) printed
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import exact, wls

pytestmark = pytest.mark.gpu

SPMV_TOL = 1e-6


def _solver(P, **kw):
    import paper_2304_14568_amd as A
    return A.Solver(P, **kw)


@pytest.fixture(scope="module")
def tiny():
    P = synth.make_tiny(0)
    W = wls.from_problem(P)
    Hm, g0, const = wls.quadratic_form(W)
    xs, info = exact.active_set(W, H=Hm, g0=g0)
    return P, W, xs, wls.objective(W, xs)


@pytest.fixture(scope="module")
def small():
    P = synth.hn_small(1)
    W = wls.from_problem(P)
    Hm, g0, const = wls.quadratic_form(W)
    xs, info = exact.active_set(W, H=Hm, g0=g0)
    return P, W, xs, wls.objective(W, xs)


def _spmv_check(got, ref, scale, tol=SPMV_TOL):
    err = np.abs(got.astype(np.float64) - ref)
    bound = tol * scale + 1e-30
    bad = np.nonzero(err > bound)[0]
    assert bad.size == 0, f"{bad.size} entries over bound; worst ratio {np.max(err / bound):.3g}"


@pytest.mark.parametrize("fmt", ["csr", "sell"])
@pytest.mark.parametrize("tile_nnz", [0, 4096])
def test_matvec_rmatvec_parity(tiny, small, tile_nnz, fmt):
    rng = np.random.default_rng(7)
    for P, W in ((tiny[0], tiny[1]), (small[0], small[1])):
        with _solver(P, tile_nnz=tile_nnz, format=fmt, xupdate="cg") as S:
            for s in range(P.num_scen):
                v = rng.uniform(0, 1, P.n).astype(np.float32)
                _spmv_check(S.matvec(v, s), wls.matvec(W, s, v), wls.matvec_abs(W, s, v))
                t = rng.normal(size=P.m).astype(np.float32)
                _spmv_check(S.rmatvec(t, s), wls.rmatvec(W, s, t), wls.rmatvec_abs(W, s, t))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_every_pass_configuration_gives_the_same_bits(small, precision):
    """Every workgroup size (256, 512, 1024) and row pipelining of the
    chunk-row pass, with 64-bit fixed-point column sums: each row's dot is
    formed by the same lanes in the same order and the column sums are exact,
    so B_s v is the same bit for bit in every configuration, and within the
    per-entry bound of the fp64 product (for bf16 values, the bound of their
    rounding: 2.5 units of 2^-8)."""
    P, W, _, _ = small
    rng = np.random.default_rng(12)
    vs = [rng.normal(size=P.n).astype(np.float32) for _ in range(2)]
    outs = {}
    for threads in (256, 512, 1024):
        for unroll in (1, 2):
            with _solver(P, pass_threads=threads, pass_unroll=unroll, lds_acc=2, format="csr", xupdate="cg",
                         precision=precision) as S:
                cfg = S.tuning(0)
                assert (cfg["threads"], cfg["unroll"], cfg["lds_acc"], cfg["format"]) == (threads, unroll, 2, "csr")
                rho = S.rho()
                outs[(threads, unroll)] = [S.normal_apply(v, s, precision=precision)
                                           for v in vs for s in (0, P.num_scen - 1)]
    first = outs[(256, 1)]
    for key, got in outs.items():
        for a, b in zip(first, got):
            assert np.array_equal(a, b), key
    tol = SPMV_TOL if precision == "fp32" else 2.5 * 2.0 ** -8
    k = 0
    for v in vs:
        for s in (0, P.num_scen - 1):
            _spmv_check(first[k], wls.normal_apply(W, s, v, rho), wls.normal_apply_abs(W, s, v, rho), tol=tol)
            k += 1


def test_pass_configuration_chosen_per_patient(tiny, small):
    """The set-up autotuner keeps a configuration per patient of a batch, each
    one of the measured candidates, with its pass time."""
    import paper_2304_14568_amd as A
    with _solver([tiny[0], small[0]], xupdate="cg") as S:
        for p in (0, 1):
            cfg = S.tuning(p)
            assert cfg["threads"] in (256, 512, 1024)
            assert cfg["unroll"] in (1, 2)
            assert cfg["lds_acc"] in (1, 2)
            assert cfg["format"] in ("csr", "sell")
            assert cfg["pass_ms"] > 0.0
            if cfg["format"] == "sell":
                assert cfg["threads"] <= 512 and cfg["unroll"] == 1
        with pytest.raises(A.AdmmError):
            S.tuning(2)


def test_forward_configuration_tuned_per_patient_and_exact(tiny, small):
    """The forward, objective and transpose products take a configuration of
    their own per patient (the fastest forward product, chosen on the first
    such product, with either x-update).  Each row's dot is formed by the same
    lanes in the same order and the transpose product's fixed-point column
    sums are exact, so both products are the same bit for bit in every
    configuration, and within the per-entry bound of the fp64 products."""
    P, W, _, _ = small
    for xupdate in ("dense", "cg"):
        with _solver([tiny[0], P], xupdate=xupdate) as S:
            assert S.forward_config(1)["pass_ms"] == 0.0  # not chosen before the first product
            S.matvec(np.ones(P.n, dtype=np.float32), 0, patient=1)
            for p in (0, 1):
                fc = S.forward_config(p)
                assert fc["threads"] in (512, 1024) and fc["unroll"] in (1, 2) and fc["pass_ms"] > 0.0
    rng = np.random.default_rng(21)
    v = rng.uniform(0.0, 1.0, P.n).astype(np.float32)
    t = rng.normal(size=P.m).astype(np.float32)
    t[rng.uniform(size=P.m) < 0.5] *= 1e-3  # entries far below the largest
    outs = {}
    for threads in (512, 1024):
        for unroll in (1, 2):
            with _solver(P, pass_threads=threads, pass_unroll=unroll, lds_acc=2, format="csr") as S:
                assert (S.forward_config(0)["threads"], S.forward_config(0)["unroll"]) == (threads, unroll)
                outs[(threads, unroll)] = [S.matvec(v, s) for s in (0, P.num_scen - 1)] + \
                                          [S.rmatvec(t, s) for s in (0, P.num_scen - 1)]
    first = outs[(512, 1)]
    for key, got in outs.items():
        for a, b in zip(first, got):
            assert np.array_equal(a, b), key
    for k, s in enumerate((0, P.num_scen - 1)):
        _spmv_check(first[k], wls.matvec(W, s, v), wls.matvec_abs(W, s, v))
        _spmv_check(first[2 + k], wls.rmatvec(W, s, t), wls.rmatvec_abs(W, s, t))


@pytest.mark.parametrize("fmt", ["csr", "sell"])
@pytest.mark.parametrize("lds_acc", [0, 1, 2])
def test_normal_apply_parity(small, lds_acc, fmt):
    P, W, _, _ = small
    rng = np.random.default_rng(8)
    with _solver(P, lds_acc=lds_acc, tile_nnz=20000, format=fmt, xupdate="cg") as S:
        rho = S.rho()
        for s in (0, 5, P.num_scen - 1):
            v = rng.normal(size=P.n).astype(np.float32)
            got = S.normal_apply(v, s)
            ref = wls.normal_apply(W, s, v, rho)
            _spmv_check(got, ref, wls.normal_apply_abs(W, s, v, rho))


@pytest.mark.parametrize("fmt", ["csr", "sell"])
def test_gradient_objective_parity(tiny, small, fmt):
    rng = np.random.default_rng(9)
    for P, W, xs, _ in (tiny, small):
        with _solver(P, format=fmt) as S:
            for x in (xs, rng.uniform(0, 0.5, P.n)):
                x32 = x.astype(np.float32).astype(np.float64)
                g, f = S.gradient(x32)
                gr = wls.gradient(W, x32)
                scale = np.zeros(P.n)
                for s in range(W.N):
                    r_abs = np.abs(W.A[s]) @ x32 + W.p
                    scale += 2 * W.c[s] * (abs(W.A[s]).T @ (W.w * r_abs))
                _spmv_check(g, gr, scale)
                fr = wls.objective(W, x32)
                assert abs(f - fr) <= 1e-6 * fr
                assert abs(S.objective(x32) - fr) <= 1e-6 * fr


@pytest.mark.parametrize("xupdate,fmt", [("cg", "csr"), ("cg", "sell"), ("dense", "auto")])
def test_admm_solve_tiny(tiny, xupdate, fmt):
    P, W, xs, fs = tiny
    with _solver(P, max_iter=3000, xupdate=xupdate, format=fmt) as S:
        zs, info, st = S.solve()
        z = zs[0]
        assert st == 0, info
        f = wls.objective(W, z)
        assert abs(f - fs) <= 1e-5 * fs
        assert abs(info[0]["obj"] - f) <= 1e-6 * fs
        assert S.kkt(z) <= 1e-3


@pytest.mark.parametrize("xupdate", ["cg", "dense"])
def test_admm_solve_hn_small(small, xupdate):
    """Paper stop: objective within 1e-5 of f*.  Residual tolerances 1e-7: the
    solver's own stop reaches KKT <= 1e-6 and the intensities are within 1e-4
    of x* (kappa(H) of this patient printed)."""
    P, W, xs, fs = small
    Hm, _, _ = wls.quadratic_form(W)
    ev = np.linalg.eigvalsh(Hm)
    cond = ev[-1] / ev[0]
    with _solver(P, max_iter=3000, xupdate=xupdate) as S:
        zs, info, st = S.solve()
        z = zs[0]
        assert st == 0, info
        f = wls.objective(W, z)
        assert abs(f - fs) <= 1e-5 * fs, (f, fs)
    with _solver(P, max_iter=5000, xupdate=xupdate, eps_abs=1e-7, eps_rel=1e-7) as S:
        zs, info, st = S.solve()
        z = zs[0]
        assert st == 0, info
        kkt = wls.kkt_residual(W, z)
        err = np.linalg.norm(z - xs) / np.linalg.norm(xs)
        print(f"[small] {xupdate} kappa(H) {cond:.3g}: {info[0]['iter']} it, kkt {kkt:.2e}, z err {err:.2e}",
              flush=True)
        assert kkt <= 1e-6 and info[0]["kkt"] <= 1e-6
        assert err <= 1e-4, err


def test_pgd_gpu(tiny):
    P, W, xs, fs = tiny
    with _solver(P) as S:
        x, info, st = S.pgd(0, obj_rel_tol=1e-9, max_iter=5000)
        f = wls.objective(W, x)
        assert f >= fs * (1 - 1e-7)
        assert abs(f - fs) <= 1e-4 * fs


@pytest.mark.parametrize("fmt", ["csr", "sell"])
def test_fixed_point_pass_is_deterministic(small, fmt):
    """With 64-bit fixed-point column accumulators every sum in an iteration is
    order-independent or in a fixed order, so two runs agree bit for bit."""
    P = small[0]
    with _solver(P, lds_acc=2, xupdate="cg", format=fmt) as S:
        rng = np.random.default_rng(11)
        v = rng.normal(size=P.n).astype(np.float32)
        a = S.normal_apply(v, 3)
        b = S.normal_apply(v, 3)
        assert np.array_equal(a, b)
        S.iterate(6)
        z1 = S.z()
        S.reset()
        S.iterate(6)
        z2 = S.z()
        assert np.array_equal(z1, z2)


def test_layouts_agree_bit_for_bit(small):
    """The chunk-row and the sliced layouts hold the same chunks of the same
    rows, each lane takes the same chunks of its row and the row sums use the
    same lane butterfly, and the column sums are exact (64-bit fixed point):
    products and iterates agree bit for bit."""
    P = small[0]
    rng = np.random.default_rng(12)
    v = rng.normal(size=P.n).astype(np.float32)
    t = rng.normal(size=P.m).astype(np.float32)
    out = {}
    for fmt in ("csr", "sell"):
        with _solver(P, lds_acc=2, xupdate="cg", format=fmt, deterministic=1) as S:
            res = [S.matvec(v, 2), S.rmatvec(t, 2), S.normal_apply(v, 2)]
            S.iterate(5)
            res.append(S.z())
            out[fmt] = res
    for a, b in zip(out["csr"], out["sell"]):
        assert np.array_equal(a, b)
