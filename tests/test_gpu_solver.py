"""GPU solver behaviour beyond single-problem parity: several patients in one
context, reduced-precision matrix copies, large spot counts, checkpoint and
resume, graph replay.  Compared with the FP64 oracle where it is the judge."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import exact, wls

pytestmark = pytest.mark.gpu


def _fstar(P):
    W = wls.from_problem(P)
    Hm, g0, _ = wls.quadratic_form(W)
    xs, _ = exact.active_set(W, H=Hm, g0=g0)
    return W, xs, wls.objective(W, xs)


@pytest.fixture(scope="module")
def patients():
    # uneven patients: different m, n and scenario counts (13-scenario recipe and a shift lattice)
    Ps = [synth.hn_small(3), synth.make_tiny(1), synth.hn_small(4, scenarios="lattice", num_scen=9)]
    return [(P,) + _fstar(P) for P in Ps]


@pytest.mark.parametrize("xupdate", ["cg", "dense"])
def test_batched_patients_match_oracle_and_single(patients, xupdate):
    import paper_2304_14568_amd as A
    Ps = [p[0] for p in patients]
    with A.Solver(Ps, max_iter=3000, tile_nnz=16384, xupdate=xupdate) as S:
        zs, infos, st = S.solve()
        assert st == 0, infos
    for (P, W, xs, fs), z, info in zip(patients, zs, infos):
        f = wls.objective(W, z)
        assert abs(f - fs) <= 1e-5 * fs, (P.name, f, fs)
        assert abs(info["obj"] - f) <= 1e-6 * fs
        with A.Solver(P, max_iter=3000, tile_nnz=16384, xupdate=xupdate) as S1:
            z1, i1, _ = S1.solve()
        assert abs(wls.objective(W, z1[0]) - f) <= 2e-6 * fs


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_reduced_precision_reaches_fp32_objective(patients, precision):
    """bf16/fp16 values with per-row scales inside CG; the residual of every
    x-update system is recomputed with the fp32 matrix, so the fixed point is
    the fp32 problem's and the objective meets the same 1e-5 bar."""
    import paper_2304_14568_amd as A
    P, W, xs, fs = patients[0]
    with A.Solver(P, max_iter=3000, precision=precision, xupdate="cg") as S:
        zs, info, st = S.solve()
        assert st == 0, info
        f = wls.objective(W, zs[0])
        assert abs(f - fs) <= 1e-5 * fs, (precision, f, fs)
        # the reduced-precision operator itself: per-entry error of bf16/fp16 rounding
        rng = np.random.default_rng(3)
        v = rng.uniform(0, 1, P.n).astype(np.float32)
        got = S.normal_apply(v, 0, precision=precision)
        ref = wls.normal_apply(W, 0, v, S.rho())
        scale = wls.normal_apply_abs(W, 0, v, S.rho())
        # unit roundoff of the format; fp16 also flushes entries far below the
        # row maximum into its subnormal range (absolute error 2^-25 of the row scale)
        u = 2.0 ** -8 if precision == "bf16" else 2.0 ** -11
        floor = 0.0 if precision == "bf16" else 2.0 ** -20 * scale.max()
        assert np.all(np.abs(got - ref) <= 2.5 * u * scale + floor + 1e-30)


@pytest.mark.parametrize("threads", [0, 512, 1024])
def test_large_spot_count_uses_extended_lds(threads):
    """n > 5461 needs more than 64 KB of LDS for the column accumulators: one
    workgroup per CU, of 512 or 1024 threads (0: the autotuner's choice)."""
    import paper_2304_14568_amd as A
    P = synth.make_hn(seed=7, grid=(64, 64, 40), body_semi_vox=(28, 22, 16), target_size=0.8, num_layers=14,
                      spot_spacing=2.5, num_scen=2)
    assert 12 * P.n > 65536
    W = wls.from_problem(P)
    rng = np.random.default_rng(4)
    with A.Solver(P, max_iter=400, lds_acc=2, xupdate="cg", pass_threads=threads) as S:
        if threads:
            assert S.tuning(0)["threads"] == threads
        for s in range(P.num_scen):
            v = rng.normal(size=P.n).astype(np.float32)
            got = S.normal_apply(v, s)
            ref = wls.normal_apply(W, s, v, S.rho())
            assert np.all(np.abs(got - ref) <= 1e-6 * wls.normal_apply_abs(W, s, v, S.rho()) + 1e-30)
            t = rng.normal(size=P.m).astype(np.float32)
            got = S.rmatvec(t, s)
            assert np.all(np.abs(got - wls.rmatvec(W, s, t)) <= 1e-6 * wls.rmatvec_abs(W, s, t) + 1e-30)
        S.iterate(200)
        z = S.z()
        # objective decreases from f(0) and the iterate is feasible
        assert np.all(z >= 0)
        assert wls.objective(W, z) < 0.5 * wls.objective(W, np.zeros(P.n))


def test_checkpoint_resume_is_exact(patients):
    import paper_2304_14568_amd as A
    P = patients[0][0]
    with A.Solver(P, lds_acc=2, use_graph=0, xupdate="cg") as S:
        S.iterate(7)
        saved = S.get_state()
        S.iterate(9)
        za = S.z()
        S.set_state(saved)
        S.iterate(9)
        zb = S.z()
        assert np.array_equal(za, zb)
    # resume in a fresh context
    with A.Solver(P, lds_acc=2, use_graph=0, xupdate="cg") as S2:
        S2.set_state(saved)
        S2.iterate(9)
        assert np.array_equal(S2.z(), za)


@pytest.mark.parametrize("xupdate", ["cg", "dense"])
def test_graph_replay_matches_direct_launches(patients, xupdate):
    import paper_2304_14568_amd as A
    P = patients[0][0]
    out = []
    for g in (0, 1):
        with A.Solver(P, lds_acc=2, use_graph=g, xupdate=xupdate) as S:
            S.iterate(12)
            z1 = S.z()
            S.reset()
            S.iterate(12)
            assert np.array_equal(S.z(), z1)
            out.append(z1)
    assert np.array_equal(out[0], out[1])


def test_device_resident_csr_input_matches_host_input():
    """CSR arrays handed over as GPU tensors (ADMM_MEM_DEVICE) give the same
    set-up and the same iterates as the same arrays in host memory."""
    import dataclasses

    import torch

    import paper_2304_14568_amd as A
    P = synth.hn_small(2)
    dev = torch.device("cuda:0")
    Ad = [synth.Csr(row_ptr=torch.from_numpy(a.row_ptr.astype(np.int64)).to(dev),
                    col=torch.from_numpy(a.col.astype(np.int32)).to(dev),
                    val=torch.from_numpy(a.val.astype(np.float32)).to(dev)) for a in P.A]
    Pd = dataclasses.replace(P, A=Ad)
    torch.cuda.synchronize()
    with A.Solver(P, xupdate="cg", lds_acc=2) as Sh, A.Solver(Pd, xupdate="cg", lds_acc=2) as Sd:
        Sh.iterate(5)
        Sd.iterate(5)
        assert np.array_equal(Sh.z(), Sd.z())
