"""Dose-volume evaluation of plans across scenarios (Sec. 3, Table 2).

The doses A_s x of every scenario and their per-structure histograms, sums and
maxima are computed on the GPU (admm_dose_stats); this module turns them into
  * DVH curves per scenario and their bands (min / max over scenarios),
  * D98, D3, Dmax and Dmean per structure and scenario,
  * the Table 2 style criteria, scaled to the prescription p of each target:
    D98 >= 0.95 p, Dmax <= 1.10 p, D3 <= 1.07 p on targets (66.5 / 77 /
    74.9 Gy at 70 Gy), and Dmean <= limit on each organ at risk.
D_v is the highest dose that at least v percent of the structure receives;
from the histogram it is reported as the centre of the bin that holds it, so
its error is at most half a bin width (dmax / nbins / 2).  DVH values at bin
edges and Dmax / Dmean are exact for the fp32 doses.
"""
from __future__ import annotations

import math

import numpy as np

TARGET_CRITERIA = {"D98": (">=", 0.95), "Dmax": ("<=", 1.10), "D3": ("<=", 1.07)}


def _dv_from_hist(counts_desc_cum, K, v, w):
    r = max(1, int(math.ceil(v * K / 100.0 - 1e-12)))
    # counts_desc_cum[k] = number of voxels in bins >= k; find the largest k with >= r
    k = int(np.nonzero(counts_desc_cum >= r)[0].max())
    return (k + 0.5) * w


def max_bins(num_groups: int) -> int:
    """Largest histogram the GPU kernel holds in LDS for this many groups (12 G + 4 G nbins <= 64 KiB)."""
    return (65536 - 12 * num_groups) // (4 * num_groups)


def evaluate(S, P, x, patient: int = 0, nbins=None, dmax=None) -> dict:
    G = int(len(P.struct_weight))
    nbins = min(4096, max_bins(G)) if nbins is None else int(nbins)
    presc = np.asarray(P.presc, dtype=np.float64)
    dmax = float(dmax) if dmax else 2.0 * max(1e-12, presc.max())
    counts, sums, maxes, _ = S.dose_stats(x, P.struct_id, G, nbins, dmax, patient)
    N = counts.shape[0]
    w = dmax / nbins
    K = counts.sum(axis=2)                        # voxels per scenario and group
    cum = np.cumsum(counts[:, :, ::-1], axis=2)[:, :, ::-1]   # voxels in bins >= k
    with np.errstate(invalid="ignore", divide="ignore"):
        dvh = cum / K[:, :, None]
    met = {k: np.full((N, G), np.nan) for k in ("D98", "D3", "Dmax", "Dmean")}
    for s in range(N):
        for g in range(G):
            if K[s, g] == 0:
                continue
            met["D98"][s, g] = _dv_from_hist(cum[s, g], K[s, g], 98.0, w)
            met["D3"][s, g] = _dv_from_hist(cum[s, g], K[s, g], 3.0, w)
            met["Dmax"][s, g] = maxes[s, g]
            met["Dmean"][s, g] = sums[s, g] / K[s, g]
    names = P.meta.get("struct_names", [f"s{g}" for g in range(G)]) if P.meta else [f"s{g}" for g in range(G)]
    limits = P.meta.get("oar_limit", [0.0] * G) if P.meta else [0.0] * G
    crit = []
    sid = np.asarray(P.struct_id)
    for g, nm in enumerate(names):
        if nm.startswith("target"):
            pt = float(presc[sid == g].max()) if np.any(sid == g) else 0.0
            for key, (op, fac) in TARGET_CRITERIA.items():
                vals = met[key][:, g]
                ok = vals >= fac * pt if op == ">=" else vals <= fac * pt
                crit.append(dict(structure=nm, metric=key, bound=fac * pt, op=op, nominal=float(vals[0]),
                                 worst=float(vals.min() if op == ">=" else vals.max()),
                                 scenarios_met=int(np.count_nonzero(ok)), scenarios=N))
        elif nm.startswith("oar") and limits[g] > 0:
            vals = met["Dmean"][:, g]
            ok = vals <= limits[g]
            crit.append(dict(structure=nm, metric="Dmean", bound=float(limits[g]), op="<=", nominal=float(vals[0]),
                             worst=float(vals.max()), scenarios_met=int(np.count_nonzero(ok)), scenarios=N))
    levels = np.arange(nbins) * w
    return dict(names=names, levels=levels, dvh=dvh, dvh_band_min=np.nanmin(dvh, axis=0),
                dvh_band_max=np.nanmax(dvh, axis=0), dvh_nominal=dvh[0], metrics=met, criteria=crit,
                bin_width=w, counts=counts)


def criteria_table(ev: dict) -> str:
    rows = ["structure  metric  bound   nominal  worst    met"]
    for c in ev["criteria"]:
        rows.append(f"{c['structure']:<10} {c['metric']:<6} {c['op']}{c['bound']:.3f}  {c['nominal']:.4f}   "
                    f"{c['worst']:.4f}   {c['scenarios_met']}/{c['scenarios']}")
    return "\n".join(rows)
