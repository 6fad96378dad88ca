"""Parity of the batched multi-patient context in the configuration of the
batch workload: several patients in one context, 64 shift-lattice scenarios
each, bf16 values inside CG (fp32 outer residual), one launch per phase for
all patients.  The two smallest patients of the batch recipe (seed 10) are
solved together and each is compared with the oracle's exact minimiser stored
by tests/golden/make_references.py (objective 1e-5, KKT residual 1e-6, and
intensities 1e-4 at residual tolerances 1e-7)."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import wls
from tests.golden.refs import load

pytestmark = pytest.mark.gpu

PATIENTS = (2, 1)


@pytest.fixture(scope="module")
def batch():
    out = []
    for k in PATIENTS:
        P = synth.batch_patient(k, num=8, scen=64, seed=10)
        rec, xs = load(f"batch_s10_p{k}")
        assert rec is not None and rec["digest"] == P.digest(), "stored oracle minimum missing or stale"
        print(f"[batch] patient {k}: m={P.m} n={P.n} N={P.num_scen} nnz={P.nnz} kappa(H)={rec['cond_H']:.3g}",
              flush=True)
        out.append((P, wls.from_problem(P), rec["f_star"], xs, rec["cond_H"]))
    return out


@pytest.mark.parametrize("eps", [1e-6, 1e-7])
def test_batched_bf16_lattice_matches_the_oracle(batch, eps):
    import paper_2304_14568_amd as A
    with A.Solver([b[0] for b in batch], xupdate="cg", precision="bf16", max_iter=4000, eps_abs=eps,
                  eps_rel=eps) as S:
        zs, info, st = S.solve()
        assert st == 0, info
        for (P, W, fs, xs, cond), z, inf in zip(batch, zs, info):
            f = wls.objective(W, z)
            kkt = wls.kkt_residual(W, z)
            err = float(np.linalg.norm(z - xs) / np.linalg.norm(xs))
            print(f"[batch] eps {eps:g} n={P.n}: {inf['iter']} it, gap {(f - fs) / fs:.2e}, kkt {kkt:.2e} "
                  f"(library {inf['kkt']:.2e}), z err {err:.2e}", flush=True)
            assert abs(f - fs) <= 1e-5 * fs
            assert kkt <= 1e-6 and inf["kkt"] <= 1e-6
            if eps <= 1e-7:
                assert err <= 1e-4, err
