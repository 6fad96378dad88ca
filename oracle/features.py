"""FP64 reference of the dose-derived spot features of the warm start (TEST INFRASTRUCTURE).

Not part of the paper.  For spot j and scenario s, with the column a_{s,:j}
of the dose matrix (Sec. 2.1 notation) and voxel classes 0 other, 1 target,
2 organ at risk:
  T_sj = sum_{i in targets} a_sij, O_sj = sum_{i in OARs} a_sij, M_sj = sum_i a_sij
  0..2  mean / min / max over s of T_sj / M_sj   (0 where M_sj = 0)
  3..4  mean / max over s of O_sj / M_sj
  5     log(1 + mean_s M_sj)
  6     sum_s (A_s^T c_s W p)_j / sum_s (A_s^T c_s W A_s)_jj   (0 where the denominator is 0)
Each is the plain definition written out; the tests compare the GPU features
with these values.
"""
from __future__ import annotations

import numpy as np

NUM_DOSE_FEATURES = 7


def spot_features(W, voxel_class) -> np.ndarray:
    vc = np.asarray(voxel_class)
    n, N = W.n, W.N
    ft = np.zeros((N, n))
    fo = np.zeros((N, n))
    mass = np.zeros((N, n))
    bsum = np.zeros(n)
    gsum = np.zeros(n)
    for s in range(N):
        A = W.A[s]
        T = A.T @ (vc == 1).astype(np.float64)
        O = A.T @ (vc == 2).astype(np.float64)
        M = A.T @ np.ones(W.m)
        safe = np.where(M > 0, M, 1.0)
        ft[s] = np.where(M > 0, T / safe, 0.0)
        fo[s] = np.where(M > 0, O / safe, 0.0)
        mass[s] = M
        bsum += W.c[s] * (A.T @ (W.w * W.p))
        gsum += W.c[s] * np.asarray(A.multiply(A).T @ W.w).ravel()
    out = np.zeros((n, NUM_DOSE_FEATURES))
    out[:, 0] = ft.mean(axis=0)
    out[:, 1] = ft.min(axis=0)
    out[:, 2] = ft.max(axis=0)
    out[:, 3] = fo.mean(axis=0)
    out[:, 4] = fo.max(axis=0)
    out[:, 5] = np.log1p(mass.mean(axis=0))
    out[:, 6] = np.where(gsum > 0, bsum / np.where(gsum > 0, gsum, 1.0), 0.0)
    return out
