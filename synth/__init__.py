"""Seeded synthetic robust-planning problems (inputs only).

This module builds the inputs of the robust weighted least-squares problem of
Sec. 2.1 (eq. for f_s and the problem "minimize sum_s f_s(x) s.t. x >= 0"):
per-scenario dose-influence matrices A_s (voxels x spots, CSR), per-voxel
structure ids with per-structure weights w (constant within a structure, as
Sec. 2.1 states), the prescription p (D_pres on target voxels, 0 elsewhere),
spot bounds and scenario probabilities c_s (the weighted-scenario remark at the
end of Sec. 2.1).

The paper plans real head-and-neck CT cases with a clinical pencil-beam engine
and 13 scenarios built from +-3 mm setup shifts and +-3.5 % range errors
(Sec. 2.3, Table 1).  Those data are not available; every problem here is a
seeded analytic phantom of the same shape: an ellipsoidal body, irregular
targets, ellipsoidal organs at risk, coplanar beams with a 5 mm lateral spot
grid and several energy layers, and the same scenario recipe.  The heavy part,
the dose-influence matrix itself, is computed by the C routine in dose.c.

Nothing here evaluates, solves or transforms the optimisation problem: the
generator is shared by the CPU oracle and the GPU library, and holds none of
the method's arithmetic.
"""
from __future__ import annotations

import ctypes
import dataclasses
import hashlib
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dose.c")
_LIB = os.path.join(_HERE, "_dose.so")

STRUCT_NORMAL = 0


def build(force: bool = True) -> str:
    """Compile the dose generator into synth/_dose.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Csr(ctypes.Structure):
    _fields_ = [
        ("nnz", ctypes.c_int64),
        ("m", ctypes.c_int32),
        ("n", ctypes.c_int32),
        ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
        ("col", ctypes.POINTER(ctypes.c_int32)),
        ("val", ctypes.POINTER(ctypes.c_float)),
    ]


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.synth_dose_csr.restype = ctypes.c_int
        lib.synth_dose_csr.argtypes = [
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
            ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_double, ctypes.c_double, ctypes.POINTER(_Csr),
        ]
        lib.synth_csr_free.restype = None
        lib.synth_csr_free.argtypes = [ctypes.POINTER(_Csr)]
        _lib_handle = lib
    return _lib_handle


@dataclasses.dataclass
class Csr:
    """One scenario's dose-influence matrix in CSR (m rows = voxels, n cols = spots)."""
    row_ptr: np.ndarray  # int64[m+1]
    col: np.ndarray      # int32[nnz], ascending within a row
    val: np.ndarray      # float32[nnz], > 0

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


@dataclasses.dataclass
class Problem:
    """Inputs of the robust WLS problem for one synthetic patient."""
    m: int
    n: int
    A: List[Csr]                    # one per scenario
    prob: np.ndarray                # float64[N] scenario weights c_s
    struct_id: np.ndarray           # uint8[m]
    struct_weight: np.ndarray       # float64[K]
    presc: np.ndarray               # float64[m]
    lb: np.ndarray                  # float64[n]
    ub: np.ndarray                  # float64[n]
    name: str = ""
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def num_scen(self) -> int:
        return len(self.A)

    @property
    def nnz(self) -> int:
        return sum(a.nnz for a in self.A)

    def weights(self) -> np.ndarray:
        """Per-voxel weight w_i = struct_weight[struct_id[i]]."""
        return self.struct_weight[self.struct_id.astype(np.int64)]

    def digest(self) -> str:
        """Stable content hash (identifies a generated instance)."""
        h = hashlib.sha256()
        for arr in (self.struct_id, self.struct_weight, self.presc, self.lb, self.ub, self.prob):
            h.update(np.ascontiguousarray(arr).tobytes())
        for a in self.A:
            h.update(a.row_ptr.tobytes())
            h.update(a.col.tobytes())
            h.update(a.val.tobytes())
        return h.hexdigest()[:16]

    def subset(self, scen: Sequence[int]) -> "Problem":
        """The same patient restricted to a subset of scenarios."""
        return dataclasses.replace(self, A=[self.A[s] for s in scen],
                                   prob=self.prob[list(scen)].copy(),
                                   name=f"{self.name}[{len(scen)} scen]")


def dose_csr(grid: Tuple[int, int, int], h: float, row_of_voxel: np.ndarray, m: int,
             origin: np.ndarray, axis: np.ndarray, rng_mm: np.ndarray,
             sigma: float, drop_rel: float = 1e-4) -> Csr:
    """Call the C generator for one scenario and copy its CSR into numpy."""
    nx, ny, nz = grid
    rov = np.ascontiguousarray(row_of_voxel, dtype=np.int32)
    o = np.ascontiguousarray(origin, dtype=np.float64)
    a = np.ascontiguousarray(axis, dtype=np.float64)
    r = np.ascontiguousarray(rng_mm, dtype=np.float64)
    n = int(r.shape[0])
    out = _Csr()
    rc = _lib().synth_dose_csr(nx, ny, nz, h, rov.ctypes.data, m, n, o.ctypes.data,
                               a.ctypes.data, r.ctypes.data, sigma, drop_rel, ctypes.byref(out))
    if rc != 0:
        raise MemoryError(f"synth_dose_csr failed ({rc})")
    try:
        nnz = int(out.nnz)
        row_ptr = np.ctypeslib.as_array(out.row_ptr, shape=(m + 1,)).copy()
        col = np.ctypeslib.as_array(out.col, shape=(max(nnz, 1),))[:nnz].copy()
        val = np.ctypeslib.as_array(out.val, shape=(max(nnz, 1),))[:nnz].copy()
    finally:
        _lib().synth_csr_free(ctypes.byref(out))
    return Csr(row_ptr, col, val)


# ----------------------------------------------------------------------------
# geometry helpers
# ----------------------------------------------------------------------------

def _voxel_centres(grid, h):
    nx, ny, nz = grid
    ix = (np.arange(nx) + 0.5) * h
    iy = (np.arange(ny) + 0.5) * h
    iz = (np.arange(nz) + 0.5) * h
    # linear index = ix + nx*(iy + ny*iz): z slowest, x fastest
    Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def _in_ellipsoid(pts, centre, semi):
    d = (pts - np.asarray(centre)) / np.asarray(semi)
    return np.einsum("ij,ij->i", d, d) <= 1.0


def _ray_enter_ellipsoid(p0, d, centre, semi):
    """Smallest t with p0 + t d inside the ellipsoid (rows of p0), NaN when missed."""
    s = np.asarray(semi, dtype=np.float64)
    q = (p0 - np.asarray(centre)) / s
    e = np.asarray(d, dtype=np.float64) / s
    a = float(e @ e)
    b = 2.0 * (q @ e)
    c = np.einsum("ij,ij->i", q, q) - 1.0
    disc = b * b - 4 * a * c
    t = np.full(p0.shape[0], np.nan)
    ok = disc >= 0
    t[ok] = (-b[ok] - np.sqrt(disc[ok])) / (2 * a)
    return t


def _beam_frame(angle_deg: float):
    """Coplanar beam in the x-y plane: direction of travel and two lateral axes."""
    th = np.deg2rad(angle_deg)
    d = np.array([np.cos(th), np.sin(th), 0.0])
    e1 = np.array([-np.sin(th), np.cos(th), 0.0])
    e2 = np.array([0.0, 0.0, 1.0])
    return d, e1, e2


# ----------------------------------------------------------------------------
# scenario sets
# ----------------------------------------------------------------------------

def scenarios_13(shift_mm: float = 3.0, range_rel: float = 0.035):
    """Nominal, +-shift on x/y/z, range x(1-r) and x(1+r), and four combined
    shift+range cases: 13 scenarios as in Sec. 2.3.  Returns (shifts[N,3], scales[N])."""
    s = shift_mm
    lo, hi = 1.0 - range_rel, 1.0 + range_rel
    shifts = [(0, 0, 0), (s, 0, 0), (-s, 0, 0), (0, s, 0), (0, -s, 0), (0, 0, s), (0, 0, -s),
              (0, 0, 0), (0, 0, 0), (s, 0, 0), (-s, 0, 0), (0, s, 0), (0, -s, 0)]
    scales = [1.0, 1, 1, 1, 1, 1, 1, lo, hi, hi, lo, hi, lo]
    return np.asarray(shifts, dtype=np.float64), np.asarray(scales, dtype=np.float64)


def scenarios_lattice(num: int, rng: np.random.Generator, shift_mm: float = 3.0,
                      range_rel: float = 0.035):
    """Per-axis shift lattice {-s, 0, +s} on x/y/z times three range scales, with the
    zero shift counted once (7 x 3 = 21 unique), padded to `num` with uniform draws
    of shift in [-s, s]^3 and range scale in [1-r, 1+r]."""
    s = shift_mm
    base = [(0, 0, 0), (s, 0, 0), (-s, 0, 0), (0, s, 0), (0, -s, 0), (0, 0, s), (0, 0, -s)]
    shifts, scales = [], []
    for sc in (1.0, 1.0 - range_rel, 1.0 + range_rel):
        for b in base:
            shifts.append(b)
            scales.append(sc)
    shifts = shifts[:num]
    scales = scales[:num]
    extra = num - len(shifts)
    if extra > 0:
        shifts += [tuple(v) for v in rng.uniform(-s, s, size=(extra, 3))]
        scales += list(rng.uniform(1.0 - range_rel, 1.0 + range_rel, size=extra))
    return np.asarray(shifts, dtype=np.float64), np.asarray(scales, dtype=np.float64)


# ----------------------------------------------------------------------------
# tiny single-beam phantom (beam along +z)
# ----------------------------------------------------------------------------

def make_tiny(seed: int = 0, grid=(20, 20, 20), h: float = 2.0, spots=(10, 10),
              spacing: float = 3.0, target_r_vox: float = 5.0, oar_r_vox: float = 3.0,
              sigma: float = 3.0, ub: float = 10.0, num_scen: int = 3,
              range_scales=(1.0, 0.965, 1.035), jitter: float = 0.5,
              probs: Optional[Sequence[float]] = None) -> Problem:
    """All voxels are rows; one beam along +z entering at z = 0; a lateral grid
    of spots on one energy layer whose range is the target-centre depth;
    range scenarios scale that range.  Target sphere (w=1, p=1), adjacent OAR
    sphere (w=0.5, p=0, max-dose limit 0.3 for evaluation only), normal tissue
    (w=0.1).  Bounds 0 <= x <= ub."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = grid
    pts = _voxel_centres(grid, h)
    centre = np.array([nx * h / 2, ny * h / 2, nz * h / 2])
    tr = target_r_vox * h
    orr = oar_r_vox * h
    off = (tr + orr + 1.0) / np.sqrt(2.0)
    oar_c = centre + np.array([off, off, 0.0])
    tgt = np.linalg.norm(pts - centre, axis=1) <= tr
    oar = (np.linalg.norm(pts - oar_c, axis=1) <= orr) & ~tgt
    sid = np.zeros(pts.shape[0], dtype=np.uint8)
    sid[oar] = 2
    sid[tgt] = 1
    weights = np.array([0.1, 1.0, 0.5])
    presc = np.where(tgt, 1.0, 0.0)
    m = pts.shape[0]
    row_of_voxel = np.arange(m, dtype=np.int32)

    ns_x, ns_y = spots
    ux = (np.arange(ns_x) - (ns_x - 1) / 2) * spacing
    uy = (np.arange(ns_y) - (ns_y - 1) / 2) * spacing
    UY, UX = np.meshgrid(uy, ux, indexing="ij")
    lat = np.stack([UX.ravel(), UY.ravel()], axis=1) + centre[:2]
    lat = lat + rng.uniform(-jitter, jitter, size=lat.shape)
    n = lat.shape[0]
    origin = np.concatenate([lat, np.zeros((n, 1))], axis=1)
    axis = np.tile(np.array([0.0, 0.0, 1.0]), (n, 1))
    r0 = centre[2]
    scales = list(range_scales)[:num_scen]
    while len(scales) < num_scen:
        scales.append(float(rng.uniform(0.965, 1.035)))
    A = [dose_csr(grid, h, row_of_voxel, m, origin, axis, np.full(n, r0 * sc), sigma)
         for sc in scales]
    c = np.ones(num_scen) if probs is None else np.asarray(probs, dtype=np.float64)
    return Problem(m=m, n=n, A=A, prob=c, struct_id=sid, struct_weight=weights,
                   presc=presc, lb=np.zeros(n), ub=np.full(n, float(ub)),
                   name=f"tiny{grid[0]}-s{seed}",
                   meta=dict(grid=grid, h=h, oar_limit=[0.0, 0.0, 0.3],
                             struct_names=["normal", "target", "oar"],
                             range_scales=np.asarray(scales), spot_xy=lat,
                             spot_beam=np.zeros(n, dtype=np.int32),
                             spot_range=np.full(n, r0), num_beams=1))


def make_brute(seed: int, spots=(3, 4)) -> Problem:
    """Tiny instance for brute-force checks: 10^3 grid, 3 x 4 = 12 spots, 3 scenarios,
    a seeded upper bound in [0.2, 1.5] and spot spacing in [3, 5] mm so that
    different seeds bind different spots."""
    rng = np.random.default_rng(10_000 + seed)
    ub = float(rng.uniform(0.2, 1.5))
    spacing = float(rng.uniform(3.0, 5.0))
    return make_tiny(seed=seed, grid=(10, 10, 10), h=2.0, spots=spots, spacing=spacing,
                     target_r_vox=3.0, oar_r_vox=2.0, sigma=3.0, ub=ub)


# ----------------------------------------------------------------------------
# head-and-neck-shaped multi-beam phantom
# ----------------------------------------------------------------------------

def make_hn(seed: int = 0, grid=(120, 120, 80), h: float = 2.5, body_semi_vox=(50, 40, 30),
            beams=(0.0, 120.0, 240.0), num_layers: int = 15, spot_spacing: float = 5.0,
            margin: float = 4.0, sigma: float = 2.5, target_size: float = 1.05,
            num_targets: int = 2, target_presc=(1.0, 0.85), num_oars: int = 4,
            scenarios: str = "13", num_scen: int = 13, ub: float = 10.0,
            jitter: float = 0.5, drop_rel: float = 1e-4) -> Problem:
    """Ellipsoidal body, `num_targets` irregular targets (each a union of three
    random ellipsoids), `num_oars` random OAR ellipsoids, coplanar beams at
    `beams` degrees, 5 mm lateral spot grid over the targets plus `margin`,
    `num_layers` energy layers spanning the target depths of each beam.

    scenarios="13": the 13-scenario recipe (nominal, +-3 mm x/y/z, range +-3.5 %,
    four combined).  scenarios="lattice": shift lattice x range, padded to
    `num_scen` with random draws.
    Targets: w=1, p=target_presc[k]; OARs: w=0.5, p=0 (their max-dose limits,
    drawn in [0.2, 0.6], are for evaluation only); normal tissue w=0.1."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = grid
    pts = _voxel_centres(grid, h)
    centre = np.array([nx * h / 2, ny * h / 2, nz * h / 2])
    body_semi = np.asarray(body_semi_vox, dtype=np.float64) * h
    body = _in_ellipsoid(pts, centre, body_semi)
    body_idx = np.nonzero(body)[0]
    m = int(body_idx.shape[0])
    row_of_voxel = np.full(pts.shape[0], -1, dtype=np.int32)
    row_of_voxel[body_idx] = np.arange(m, dtype=np.int32)
    bp = pts[body_idx]

    sid = np.zeros(m, dtype=np.uint8)
    presc = np.zeros(m)
    tmask = np.zeros(m, dtype=bool)
    tgt_masks = []
    scale = float(target_size)
    for k in range(num_targets):
        base = centre + rng.uniform(-0.25, 0.25, size=3) * body_semi * np.array([1, 1, 0.6])
        mk = np.zeros(m, dtype=bool)
        for _ in range(3):
            c = base + rng.uniform(-8, 8, size=3) * scale
            semi = rng.uniform(9, 15, size=3) * scale
            mk |= _in_ellipsoid(bp, c, semi)
        mk &= ~tmask
        tgt_masks.append(mk)
        tmask |= mk
    oar_limits = []
    oar_masks = []
    for k in range(num_oars):
        tc = bp[tmask].mean(axis=0) if tmask.any() else centre
        dirv = rng.normal(size=3)
        dirv /= np.linalg.norm(dirv)
        c = tc + dirv * rng.uniform(20, 35) * scale
        semi = rng.uniform(6, 12, size=3) * scale
        mk = _in_ellipsoid(bp, c, semi) & ~tmask
        for prev in oar_masks:
            mk &= ~prev
        oar_masks.append(mk)
        oar_limits.append(float(rng.uniform(0.2, 0.6)))
    for k, mk in enumerate(oar_masks):
        sid[mk] = 1 + num_targets + k
    for k, mk in enumerate(tgt_masks):
        sid[mk] = 1 + k
        presc[mk] = target_presc[k % len(target_presc)]
    weights = np.array([0.1] + [1.0] * num_targets + [0.5] * num_oars)
    names = ["normal"] + [f"target{k}" for k in range(num_targets)] + [f"oar{k}" for k in range(num_oars)]

    # spot placement per beam
    iso = bp[tmask].mean(axis=0)
    tp = bp[tmask]
    half = spot_spacing / 2 + margin
    spot_beam, spot_uv, spot_R = [], [], []
    for b, ang in enumerate(beams):
        d, e1, e2 = _beam_frame(ang)
        rel = tp - iso
        u = rel @ e1
        v = rel @ e2
        t = rel @ d
        iu = np.arange(np.floor((u.min() - margin) / spot_spacing), np.ceil((u.max() + margin) / spot_spacing) + 1)
        iv = np.arange(np.floor((v.min() - margin) / spot_spacing), np.ceil((v.max() + margin) / spot_spacing) + 1)
        cand = []
        for a_ in iu:
            for b_ in iv:
                uc, vc = a_ * spot_spacing, b_ * spot_spacing
                sel = (np.abs(u - uc) <= half) & (np.abs(v - vc) <= half)
                if not sel.any():
                    continue
                cand.append((uc, vc, t[sel].min() - margin, t[sel].max() + margin))
        cand = np.asarray(cand)
        p0 = iso + cand[:, 0:1] * e1 + cand[:, 1:2] * e2 - 500.0 * d
        tin = _ray_enter_ellipsoid(p0, d, centre, body_semi) - 500.0
        dmin = cand[:, 2] - tin
        dmax = cand[:, 3] - tin
        R = np.linspace(dmin.min(), dmax.max(), num_layers)
        dl = (R[1] - R[0]) if num_layers > 1 else 1.0
        for ci in range(cand.shape[0]):
            for Rl in R:
                if dmin[ci] - dl / 2 <= Rl <= dmax[ci] + dl / 2:
                    spot_beam.append(b)
                    spot_uv.append((cand[ci, 0], cand[ci, 1]))
                    spot_R.append(Rl)
    spot_beam = np.asarray(spot_beam, dtype=np.int32)
    spot_uv = np.asarray(spot_uv, dtype=np.float64)
    spot_uv = spot_uv + rng.uniform(-jitter, jitter, size=spot_uv.shape)
    spot_R = np.asarray(spot_R, dtype=np.float64)
    n = int(spot_beam.shape[0])

    if scenarios == "13":
        shifts, scales = scenarios_13()
        shifts, scales = shifts[:num_scen], scales[:num_scen]
    else:
        shifts, scales = scenarios_lattice(num_scen, rng)

    frames = [_beam_frame(a) for a in beams]
    D = np.stack([frames[b][0] for b in spot_beam])
    E1 = np.stack([frames[b][1] for b in spot_beam])
    E2 = np.stack([frames[b][2] for b in spot_beam])
    A = []
    for s in range(shifts.shape[0]):
        q = iso + shifts[s] + spot_uv[:, 0:1] * E1 + spot_uv[:, 1:2] * E2
        p0 = q - 500.0 * D
        tin = np.empty(n)
        for b in range(len(beams)):
            sel = spot_beam == b
            tin[sel] = _ray_enter_ellipsoid(p0[sel], frames[b][0], centre, body_semi)
        origin = p0 + tin[:, None] * D
        A.append(dose_csr(grid, h, row_of_voxel, m, origin, D, spot_R * scales[s], sigma, drop_rel))
    return Problem(m=m, n=n, A=A, prob=np.ones(len(A)), struct_id=sid, struct_weight=weights,
                   presc=presc, lb=np.zeros(n), ub=np.full(n, float(ub)),
                   name=f"hn{grid[0]}x{grid[1]}x{grid[2]}-s{seed}",
                   meta=dict(grid=grid, h=h, struct_names=names,
                             oar_limit=[0.0] * (1 + num_targets) + oar_limits,
                             shifts=shifts, range_scales=scales, spot_beam=spot_beam,
                             spot_uv=spot_uv, spot_range=spot_R, num_beams=len(beams),
                             iso=iso, beam_angles=np.asarray(beams), voxel_xyz=bp))


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

def hn_full(seed: int = 0, **kw) -> Problem:
    """Head-and-neck-shaped workload: 120x120x80 grid at 2.5 mm, ~250k body voxels,
    3 coplanar beams, 15 energy layers, ~3000 spots, 13 scenarios."""
    return make_hn(seed=seed, **kw)


def hn_small(seed: int = 0, num_scen: int = 13, **kw) -> Problem:
    """A scaled-down head-and-neck phantom (same recipe) sized for the CPU oracle."""
    args = dict(grid=(48, 48, 32), body_semi_vox=(20, 16, 12), target_size=0.45,
                num_layers=8, num_scen=num_scen)
    args.update(kw)
    return make_hn(seed=seed, **args)


def batch_params(num: int, seed: int):
    """Per-patient recipe of the multi-patient batch: for patient k the linear
    body scale f ~ U[0.62, 1.17] (in-body voxels ~ f^3 * 250k, 60k..400k) and
    the target scale ~ U[0.7, 2.0], drawn in that order from one seeded stream."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(num):
        f = rng.uniform(0.62, 1.17)
        ts = rng.uniform(0.7, 2.0)
        semi = (int(50 * f), int(40 * f), int(30 * f))
        grid = (int(2 * semi[0] + 20), int(2 * semi[1] + 40), int(2 * semi[2] + 20))
        out.append(dict(seed=seed * 100 + k, grid=grid, body_semi_vox=semi, target_size=ts))
    return out


def batch_patient(k: int, num: int = 8, scen: int = 64, seed: int = 10) -> Problem:
    """Patient k of the batch recipe (batch_params) with the shift-lattice
    scenario set of `scen` scenarios."""
    p = batch_params(num, seed)[k]
    return make_hn(seed=p["seed"], grid=p["grid"], body_semi_vox=p["body_semi_vox"], target_size=p["target_size"],
                   scenarios="lattice", num_scen=scen)
