"""Pins of the dose-volume definitions and of the histogram-based evaluator's host logic (CPU)."""
from __future__ import annotations

import numpy as np

from oracle import clinical as oc


def test_dose_volume_on_integers():
    d = np.arange(1, 101, dtype=np.float64)  # 100 voxels, doses 1..100
    rng = np.random.default_rng(0)
    rng.shuffle(d)
    # 98 % of the voxels receive at least 3; 3 % receive at least 98
    assert oc.dose_volume(d, 98.0) == 3.0
    assert oc.dose_volume(d, 3.0) == 98.0
    assert oc.dose_volume(d, 100.0) == 1.0
    assert oc.dose_volume(d, 1.0) == 100.0
    # ceil rule with a volume that is not a multiple of 100: K = 7, v = 98 -> r = 7 (the minimum)
    assert oc.dose_volume(np.array([5, 1, 4, 2, 7, 3, 6.0]), 98.0) == 1.0


def test_dvh_properties():
    rng = np.random.default_rng(1)
    d = rng.gamma(4.0, 0.25, size=1000)
    lv = np.linspace(0, 3, 61)
    h = oc.dvh(d, lv)
    assert h[0] == 1.0 and np.all(np.diff(h) <= 0)
    # DVH at D_v is at least v percent
    for v in (2.0, 50.0, 98.0):
        assert oc.dvh(d, [oc.dose_volume(d, v)])[0] >= v / 100.0


def test_uniform_dose_metrics():
    D = np.full((2, 10), 0.7)
    g = np.array([0] * 4 + [1] * 6)
    m = oc.structure_metrics(D, g, 3)
    for k in ("D98", "D3", "Dmax", "Dmean"):
        assert np.allclose(m[k][:, :2], 0.7)
        assert np.all(np.isnan(m[k][:, 2]))


def test_histogram_dose_volume_within_half_bin():
    """The evaluator's histogram rule (bin holding the r-th largest dose,
    reported at its centre) against the sorted definition."""
    from paper_2304_14568_amd.clinical import _dv_from_hist
    rng = np.random.default_rng(2)
    nb, dmax = 512, 2.0
    w = dmax / nb
    for K in (1, 7, 100, 5000):
        d = rng.uniform(0, 1.9, size=K)
        counts = np.bincount(np.minimum((d / w).astype(int), nb - 1), minlength=nb)
        cum = np.cumsum(counts[::-1])[::-1]
        for v in (3.0, 50.0, 98.0):
            assert abs(_dv_from_hist(cum, K, v, w) - oc.dose_volume(d, v)) <= w / 2 + 1e-12
