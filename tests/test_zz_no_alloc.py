"""The allocation-free dose statistics (admm_dose_stats_noalloc) against the
allocating entry point admm_dose_stats, through the C ABI: two calls in a row
on one GPU, the second with a smaller input (another patient of the same
context with fewer voxels, groups and bins), so that what the first call left
in the shared scratch must not leak into the second."""
from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _same(a, b):
    ca, sa, ma, da = a
    cb, sb, mb, db = b
    assert np.array_equal(ca, cb)
    assert np.array_equal(ma, mb)
    assert np.array_equal(da, db)
    # per-group sums are fp64 atomics: equal up to the order of the additions
    assert np.all(np.abs(sa - sb) <= 1e-12 * np.maximum(1.0, np.abs(sb)))


def test_noalloc_dose_stats_match_the_allocating_entry_point():
    import paper_2304_14568_amd as A
    big, small = synth.hn_small(5), synth.make_tiny(0)
    assert small.m < big.m
    rng = np.random.default_rng(31)
    with A.Solver([big, small], xupdate="cg") as S:
        cases = [(0, big, len(big.struct_weight), 512, 1.6), (1, small, 2, 64, 2.0)]
        for patient, P, G, nb, dmax in cases:
            print(f"[noalloc] patient {patient} m={P.m} n={P.n} N={P.num_scen} G={G} nbins={nb}", flush=True)
            x = rng.uniform(0.0, 1.0, P.n)
            grp = (P.struct_id % G).astype(np.uint8)
            got = S.dose_stats(x, grp, G, nb, dmax, patient=patient, want_dose=True, noalloc=True)
            ref = S.dose_stats(x, grp, G, nb, dmax, patient=patient, want_dose=True)
            _same(got, ref)
            assert got[0].sum() == P.num_scen * P.m
