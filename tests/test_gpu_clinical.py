"""GPU dose statistics (admm_dose_stats) and the dose-volume evaluation
against the FP64 dose definitions."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from oracle import clinical as oc, exact, wls

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def plan():
    P = synth.hn_small(5)
    W = wls.from_problem(P)
    Hm, g0, _ = wls.quadratic_form(W)
    xs, _ = exact.active_set(W, H=Hm, g0=g0)
    return P, W, xs


def test_dose_stats_parity(plan):
    import paper_2304_14568_amd as A
    P, W, xs = plan
    G, nb, dmax = len(P.struct_weight), 1024, 1.6
    with A.Solver(P) as S:
        counts, sums, maxes, dose = S.dose_stats(xs, P.struct_id, G, nb, dmax, want_dose=True)
    Dref = oc.doses(W, xs.astype(np.float32).astype(np.float64))
    x32 = xs.astype(np.float32).astype(np.float64)
    inv_w = np.float32(nb / dmax)
    for s in range(P.num_scen):
        scale = abs(W.A[s]) @ np.abs(x32)
        assert np.all(np.abs(dose[s] - Dref[s]) <= 1e-6 * scale + 1e-30)
        # the histogram of the GPU's own doses, binned as documented (fp32 product, truncation)
        b = np.minimum((dose[s] * inv_w).astype(np.int64), nb - 1)
        b[dose[s] < 0] = 0
        for g in range(G):
            sel = P.struct_id == g
            assert np.array_equal(counts[s, g], np.bincount(b[sel], minlength=nb)[:nb])
            if sel.any():
                assert maxes[s, g] == dose[s][sel].max()
                ref = float(np.sum(dose[s][sel].astype(np.float64)))
                assert abs(sums[s, g] - ref) <= 1e-12 * max(1.0, abs(ref))
            else:
                assert maxes[s, g] == -np.inf and counts[s, g].sum() == 0


def test_clinical_metrics_match_definitions(plan):
    import paper_2304_14568_amd as A
    from paper_2304_14568_amd import clinical
    P, W, xs = plan
    with A.Solver(P) as S:
        ev = clinical.evaluate(S, P, xs)
    Dref = oc.doses(W, xs)
    ref = oc.structure_metrics(Dref, P.struct_id, len(P.struct_weight))
    w = ev["bin_width"]
    for key, tol in (("D98", w / 2 + 1e-5), ("D3", w / 2 + 1e-5), ("Dmax", 1e-5), ("Dmean", 1e-6)):
        got, r = ev["metrics"][key], ref[key]
        assert np.array_equal(np.isnan(got), np.isnan(r))
        ok = ~np.isnan(r)
        assert np.all(np.abs(got[ok] - r[ok]) <= tol * np.maximum(1.0, np.abs(r[ok]))), key
    # DVH at the bin edges: fraction of voxels with dose >= edge (allow voxels within
    # fp32 rounding of an edge to fall either side)
    levels = ev["levels"][::32]
    for s in (0, P.num_scen - 1):
        for g in range(len(P.struct_weight)):
            sel = P.struct_id == g
            if not sel.any():
                continue
            d = Dref[s, sel]
            near = np.array([np.count_nonzero(np.abs(d - L) <= 1e-6 * max(L, 1e-12)) for L in levels]) / d.size
            assert np.all(np.abs(ev["dvh"][s, g, ::32] - oc.dvh(d, levels)) <= near + 1e-12)
    assert any(c["structure"].startswith("target") for c in ev["criteria"])
