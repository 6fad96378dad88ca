"""Dose-volume metrics of a plan, plain definitions (TEST INFRASTRUCTURE).

Sec. 3 judges plans by dose-volume histograms across the scenarios and by the
criteria of Table 2 (target D98% from below, target Dmax and D3% and organ
Dmax or Dmean from above).  Definitions used here, for the doses d of the K
voxels of one structure in one scenario:
  DVH(level)  fraction of the K voxels with dose >= level
  D_v         with the doses sorted in decreasing order s_1 >= ... >= s_K,
              D_v = s_r, r = ceil(v K / 100): the highest dose that at least
              v percent of the structure receives
  Dmax, Dmean maximum and mean of d
"""
from __future__ import annotations

import math

import numpy as np


def doses(W, x) -> np.ndarray:
    """d_s = A_s x for every scenario (FP64), N x m."""
    x = np.asarray(x, dtype=np.float64)
    return np.stack([W.A[s] @ x for s in range(W.N)])


def dose_volume(d, v: float) -> float:
    d = np.sort(np.asarray(d, dtype=np.float64))[::-1]
    r = max(1, int(math.ceil(v * d.size / 100.0 - 1e-12)))
    return float(d[r - 1])


def dvh(d, levels) -> np.ndarray:
    d = np.asarray(d, dtype=np.float64)
    return np.array([np.count_nonzero(d >= L) / d.size for L in np.asarray(levels, dtype=np.float64)])


def structure_metrics(D, groups, G: int) -> dict:
    """Per scenario and group: D98, D3, Dmax, Dmean (NaN for an empty group)."""
    N = D.shape[0]
    out = {k: np.full((N, G), np.nan) for k in ("D98", "D3", "Dmax", "Dmean")}
    groups = np.asarray(groups)
    for s in range(N):
        for g in range(G):
            d = D[s, groups == g]
            if d.size == 0:
                continue
            out["D98"][s, g] = dose_volume(d, 98.0)
            out["D3"][s, g] = dose_volume(d, 3.0)
            out["Dmax"][s, g] = d.max()
            out["Dmean"][s, g] = d.mean()
    return out
