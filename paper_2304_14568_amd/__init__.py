"""MI355X-native ADMM-BB for robust proton treatment planning (Fu, Taasti, Zarepisheh).

Python binding of the C-ABI library libadmmbb.so (include/admmbb.h).  This module
only marshals arguments: every step of the method runs in the library's HIP
kernels.  If the compiled library is missing, importing the binding raises; there
is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadmmbb.so")

OK, MAX_ITER = 0, 1
E_ARG, E_CSR, E_NEGATIVE, E_NONFINITE, E_OOM, E_HIP, E_DIVERGED, E_STATE = -1, -2, -3, -4, -5, -6, -7, -8
PREC = {"fp32": 0, "bf16": 1, "fp16": 2}
XUPDATE = {"auto": -1, "cg": 0, "dense": 1}
FORMAT = {"auto": -1, "csr": 0, "sell": 1}

# every symbol include/admmbb.h declares
EXPORTS = [
    "admm_default_options", "pgd_default_options", "admm_setup", "admm_setup_batch", "admm_warm_start",
    "admm_reset", "admm_iterate", "admm_solve", "pgd_solve", "admm_objective", "admm_gradient", "admm_kkt",
    "admm_matvec", "admm_rmatvec", "admm_normal_apply", "admm_get_rho", "admm_get_z", "admm_get_state",
    "admm_set_state", "admm_get_trace", "admm_get_cg_counts", "admm_get_tuning", "admm_get_pass_config", "admm_get_forward_config", "admm_get_format", "admm_get_sizes", "admm_enable_timing", "admm_get_timing",
    "admm_last_error", "admm_destroy", "admm_validate", "admm_spot_features", "admm_dose_stats", "admm_get_xupdate", "admm_time_pass",
    "admm_stream_probe", "admm_dose_stats_noalloc",
    "mlp_create", "mlp_destroy", "mlp_num_params", "mlp_get_params", "mlp_set_params", "mlp_forward",
    "mlp_loss_grad", "mlp_adam_step", "mlp_last_error",
]
NUM_DOSE_FEATURES = 7


class AdmmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"admmbb error {code}: {msg}")
        self.code = code


class CsrC(ctypes.Structure):
    _fields_ = [("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("prob", ctypes.c_double)]


class ProblemC(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("num_scen", ctypes.c_int32),
                ("A", ctypes.POINTER(CsrC)), ("struct_id", ctypes.c_void_p), ("num_struct", ctypes.c_int32),
                ("struct_weight", ctypes.c_void_p), ("presc", ctypes.c_void_p), ("lb", ctypes.c_void_p),
                ("ub", ctypes.c_void_p), ("mem_kind", ctypes.c_int32)]

MEM_HOST, MEM_DEVICE = 0, 1


class OptionsC(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("eps_abs", ctypes.c_double), ("eps_rel", ctypes.c_double),
                ("obj_rel_tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("bb", ctypes.c_int32),
                ("z_mode", ctypes.c_int32), ("bb_clamp", ctypes.c_double), ("cg_max", ctypes.c_int32),
                ("cg_eta", ctypes.c_double), ("cg_eta_floor", ctypes.c_double), ("precision", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("lds_acc", ctypes.c_int32), ("tile_nnz", ctypes.c_int32), ("pass_threads", ctypes.c_int32),
                ("pass_unroll", ctypes.c_int32), ("xupdate", ctypes.c_int32), ("format", ctypes.c_int32),
                ("deterministic", ctypes.c_int32), ("dense_launches", ctypes.c_int32),
                ("stream", ctypes.c_void_p)]


class InfoC(ctypes.Structure):
    _fields_ = [("iter", ctypes.c_int32), ("cg_steps", ctypes.c_int32), ("status", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("obj", ctypes.c_double), ("r_prim", ctypes.c_double),
                ("r_dual", ctypes.c_double), ("eps_prim", ctypes.c_double), ("eps_dual", ctypes.c_double),
                ("tau", ctypes.c_double), ("kkt", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


class PgdOptionsC(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("obj_rel_tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("max_trials", ctypes.c_int32),
                ("dense", ctypes.c_int32), ("reserved", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          f"python paper_2304_14568_amd/build.py")
    # With PyTorch installed, its HIP runtime is loaded first so that torch and
    # the library share one runtime in the process (a torch stream can then be
    # handed to the library, and neither initialises the device behind the other).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "admm_default_options": [ctypes.POINTER(OptionsC)],
        "pgd_default_options": [ctypes.POINTER(PgdOptionsC)],
        "admm_setup": [ctypes.POINTER(ProblemC), ctypes.POINTER(OptionsC), ctypes.POINTER(P)],
        "admm_setup_batch": [ctypes.POINTER(ProblemC), i32, ctypes.POINTER(OptionsC), ctypes.POINTER(P)],
        "admm_warm_start": [P, i32, P, dbl, i32],
        "admm_spot_features": [P, i32, P, P],
        "admm_dose_stats": [P, i32, P, P, i32, i32, dbl, P, P, P, P],
        "admm_dose_stats_noalloc": [P, i32, P, P, i32, i32, dbl, P, P, P, P],
        "admm_get_xupdate": [P, P, P],
        "admm_time_pass": [P, i32, i32, P],
        "admm_stream_probe": [i64, i32, P],
        "mlp_create": [i32, i32, ctypes.c_uint64, P, ctypes.POINTER(P)],
        "mlp_get_params": [P, P],
        "mlp_set_params": [P, P],
        "mlp_forward": [P, P, i32, i32, P, P],
        "mlp_loss_grad": [P, P, P, i32, ctypes.c_float, ctypes.c_float, P, P],
        "mlp_adam_step": [P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float],
        "admm_reset": [P],
        "admm_iterate": [P, i32, P],
        "admm_solve": [P, P, P],
        "pgd_solve": [P, ctypes.POINTER(PgdOptionsC), i32, P, P, P],
        "admm_objective": [P, i32, P, P],
        "admm_gradient": [P, i32, P, P, P],
        "admm_kkt": [P, i32, P, P],
        "admm_matvec": [P, i32, i32, P, P],
        "admm_rmatvec": [P, i32, i32, P, P],
        "admm_normal_apply": [P, i32, i32, i32, P, P],
        "admm_get_rho": [P, i32, P],
        "admm_get_z": [P, i32, P],
        "admm_get_state": [P, i32, P, P, P, P],
        "admm_set_state": [P, i32, P, P, P, P],
        "admm_get_trace": [P, i32, P, i32, P],
        "admm_get_cg_counts": [P, i32, P],
        "admm_get_tuning": [P, P, P, P, P],
        "admm_get_pass_config": [P, i32, P, P, P, P, P],
        "admm_get_forward_config": [P, i32, P, P, P],
        "admm_get_format": [P, P],
        "admm_get_sizes": [P, i32, P, P, P, P],
        "admm_enable_timing": [P, i32],
        "admm_get_timing": [P, P, P, P],
        "admm_validate": [ctypes.POINTER(ProblemC)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.admm_last_error.argtypes = [P]
    lib.admm_last_error.restype = ctypes.c_char_p
    lib.admm_destroy.argtypes = [P]
    lib.admm_destroy.restype = None
    lib.mlp_destroy.argtypes = [P]
    lib.mlp_destroy.restype = None
    lib.mlp_num_params.argtypes = [P]
    lib.mlp_num_params.restype = ctypes.c_int64
    lib.mlp_last_error.argtypes = []
    lib.mlp_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class _ProblemHold:
    """Keeps the contiguous numpy arrays alive while a ProblemC points at them."""

    def __init__(self, prob):
        self.arrays = []
        A = prob.A
        self.csr = (CsrC * len(A))()
        # CSR arrays given as GPU tensors (row_ptr int64, col int32, val float32,
        # contiguous) are passed as device pointers (ADMM_MEM_DEVICE)
        dev = [bool(getattr(x, "is_cuda", False)) for a in A for x in (a.row_ptr, a.col, a.val)]
        if any(dev) and not all(dev):
            raise ValueError("either every CSR array is a GPU tensor or none is")
        self.mem_kind = MEM_DEVICE if dev and all(dev) else MEM_HOST
        for s, a in enumerate(A):
            c = float(prob.prob[s]) if getattr(prob, "prob", None) is not None else 1.0
            if self.mem_kind == MEM_DEVICE:
                ptrs = []
                for x, dt in ((a.row_ptr, "int64"), (a.col, "int32"), (a.val, "float32")):
                    if str(x.dtype) != "torch." + dt or not x.is_contiguous():
                        raise ValueError(f"device CSR arrays must be contiguous torch.{dt} tensors")
                    self.arrays.append(x)
                    ptrs.append(x.data_ptr())
                self.csr[s] = CsrC(int(a.col.shape[0]), ptrs[0], ptrs[1], ptrs[2], c)
                continue
            rp = self._keep(a.row_ptr, np.int64)
            col = self._keep(a.col, np.int32)
            val = self._keep(a.val, np.float32)
            self.csr[s] = CsrC(int(col.shape[0]), rp.ctypes.data, col.ctypes.data, val.ctypes.data, c)
        sid = self._keep(prob.struct_id, np.uint8)
        sw = self._keep(prob.struct_weight, np.float64)
        pr = self._keep(prob.presc, np.float64)
        lb = None if getattr(prob, "lb", None) is None else self._keep(prob.lb, np.float64)
        ub = None if getattr(prob, "ub", None) is None else self._keep(prob.ub, np.float64)
        self.c = ProblemC(int(prob.m), int(prob.n), len(A), self.csr, sid.ctypes.data, int(sw.shape[0]),
                          sw.ctypes.data, pr.ctypes.data, _ptr(lb), _ptr(ub), self.mem_kind)

    def _keep(self, a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        self.arrays.append(a)
        return a


def _check(ctx, code: int):
    if code < 0:
        raise AdmmError(code, lib.admm_last_error(ctx).decode(errors="replace"))
    return code


def stream_probe(nbytes: int, reps: int = 10) -> float:
    """GB/s of one streaming read pass over a device buffer of nbytes;
    see admm_stream_probe."""
    gbs = ctypes.c_double()
    code = lib.admm_stream_probe(int(nbytes), int(reps), ctypes.byref(gbs))
    if code < 0:
        raise AdmmError(code, "admm_stream_probe failed")
    return gbs.value


def default_options(**kw) -> OptionsC:
    o = OptionsC()
    lib.admm_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PREC[v]
        if k == "xupdate" and isinstance(v, str):
            v = XUPDATE[v]
        if k == "format" and isinstance(v, str):
            v = FORMAT[v]
        if k == "stream" and v is not None and not isinstance(v, int):
            v = int(getattr(v, "cuda_stream", v))  # torch.cuda.Stream -> hipStream_t
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def validate(prob) -> int:
    """Host-only validation (no device needed); returns the status code."""
    h = _ProblemHold(prob)
    return lib.admm_validate(ctypes.byref(h.c))


def last_setup_error() -> str:
    return lib.admm_last_error(None).decode(errors="replace")


class Solver:
    """One context of the library over one or several patients."""

    def __init__(self, problems, **opts):
        if not isinstance(problems, (list, tuple)):
            problems = [problems]
        self.problems = list(problems)
        self._holds = [_ProblemHold(p) for p in self.problems]
        arr = (ProblemC * len(self._holds))(*[h.c for h in self._holds])
        self.opts = default_options(**opts)
        ctx = ctypes.c_void_p()
        code = lib.admm_setup_batch(arr, len(self._holds), ctypes.byref(self.opts), ctypes.byref(ctx))
        if code != OK:
            raise AdmmError(code, last_setup_error())
        self.ctx = ctx
        self._holds = None  # the library copied everything it needs
        self.n = [int(p.n) for p in self.problems]
        self.m = [int(p.m) for p in self.problems]
        self.num_scen = [len(p.A) for p in self.problems]

    def close(self):
        if getattr(self, "ctx", None):
            lib.admm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def num_patients(self) -> int:
        return len(self.problems)

    def solve(self):
        """Returns (list of z per patient, list of info dicts, status)."""
        z = np.zeros(sum(self.n))
        info = (InfoC * self.num_patients)()
        st = _check(self.ctx, lib.admm_solve(self.ctx, z.ctypes.data, info))
        out, o = [], 0
        for n in self.n:
            out.append(z[o:o + n].copy())
            o += n
        return out, [i.as_dict() for i in info], st

    def iterate(self, k: int):
        info = (InfoC * self.num_patients)()
        _check(self.ctx, lib.admm_iterate(self.ctx, int(k), info))
        return [i.as_dict() for i in info]

    def reset(self):
        _check(self.ctx, lib.admm_reset(self.ctx))

    def warm_start(self, patient: int, z0: Optional[np.ndarray] = None, rho: float = 0.0, dual_init: bool = False):
        z = None if z0 is None else np.ascontiguousarray(z0, dtype=np.float64)
        _check(self.ctx, lib.admm_warm_start(self.ctx, patient, _ptr(z), float(rho), 1 if dual_init else 0))

    def spot_features(self, voxel_class, patient: int = 0):
        """Dose-derived per-spot features (n x NUM_DOSE_FEATURES), computed on the GPU."""
        vc = np.ascontiguousarray(voxel_class, dtype=np.uint8)
        out = np.zeros((self.n[patient], NUM_DOSE_FEATURES), dtype=np.float32)
        _check(self.ctx, lib.admm_spot_features(self.ctx, patient, vc.ctypes.data, out.ctypes.data))
        return out

    def dose_stats(self, x, voxel_group, num_groups: int, nbins: int, dmax: float, patient: int = 0,
                   want_dose: bool = False, noalloc: bool = False):
        """Per-scenario, per-group dose histograms, sums and maxima of plan x
        (computed on the GPU); returns (counts[N,G,nbins], sums[N,G], maxes[N,G], doses[N,m] or None).
        noalloc: call admm_dose_stats_noalloc (fixed device scratch, no allocation)."""
        N, m = self.num_scen[patient], self.m[patient]
        xa = np.ascontiguousarray(x, dtype=np.float64)
        grp = np.ascontiguousarray(voxel_group, dtype=np.uint8)
        counts = np.zeros((N, num_groups, nbins), dtype=np.uint32)
        sums = np.zeros((N, num_groups))
        maxes = np.zeros((N, num_groups), dtype=np.float32)
        dose = np.zeros((N, m), dtype=np.float32) if want_dose else None
        fn = lib.admm_dose_stats_noalloc if noalloc else lib.admm_dose_stats
        _check(self.ctx, fn(self.ctx, patient, xa.ctypes.data, grp.ctypes.data, int(num_groups), int(nbins),
                            float(dmax), counts.ctypes.data, sums.ctypes.data, maxes.ctypes.data, _ptr(dose)))
        return counts, sums, maxes, dose

    def pgd(self, patient: int = 0, x0: Optional[np.ndarray] = None, **kw):
        o = PgdOptionsC()
        lib.pgd_default_options(ctypes.byref(o))
        for k, v in kw.items():
            if k == "dense" and isinstance(v, str):
                v = {"auto": -1, "sparse": 0, "dense": 1}[v]
            setattr(o, k, v)
        x = np.zeros(self.n[patient])
        x0a = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        info = InfoC()
        st = _check(self.ctx, lib.pgd_solve(self.ctx, ctypes.byref(o), patient, _ptr(x0a), x.ctypes.data,
                                            ctypes.byref(info)))
        return x, info.as_dict(), st

    def objective(self, x, patient: int = 0) -> float:
        xa = np.ascontiguousarray(x, dtype=np.float64)
        f = ctypes.c_double()
        _check(self.ctx, lib.admm_objective(self.ctx, patient, xa.ctypes.data, ctypes.byref(f)))
        return f.value

    def gradient(self, x, patient: int = 0):
        xa = np.ascontiguousarray(x, dtype=np.float64)
        g = np.zeros(self.n[patient])
        f = ctypes.c_double()
        _check(self.ctx, lib.admm_gradient(self.ctx, patient, xa.ctypes.data, g.ctypes.data, ctypes.byref(f)))
        return g, f.value

    def kkt(self, x, patient: int = 0) -> float:
        xa = np.ascontiguousarray(x, dtype=np.float64)
        r = ctypes.c_double()
        _check(self.ctx, lib.admm_kkt(self.ctx, patient, xa.ctypes.data, ctypes.byref(r)))
        return r.value

    def matvec(self, v, scen: int, patient: int = 0):
        va = np.ascontiguousarray(v, dtype=np.float32)
        out = np.zeros(self.m[patient], dtype=np.float32)
        _check(self.ctx, lib.admm_matvec(self.ctx, patient, scen, va.ctypes.data, out.ctypes.data))
        return out

    def rmatvec(self, t, scen: int, patient: int = 0):
        ta = np.ascontiguousarray(t, dtype=np.float32)
        out = np.zeros(self.n[patient], dtype=np.float32)
        _check(self.ctx, lib.admm_rmatvec(self.ctx, patient, scen, ta.ctypes.data, out.ctypes.data))
        return out

    def normal_apply(self, v, scen: int, patient: int = 0, precision="fp32"):
        va = np.ascontiguousarray(v, dtype=np.float32)
        out = np.zeros(self.n[patient], dtype=np.float32)
        pr = PREC[precision] if isinstance(precision, str) else int(precision)
        _check(self.ctx, lib.admm_normal_apply(self.ctx, patient, scen, pr, va.ctypes.data, out.ctypes.data))
        return out

    def rho(self, patient: int = 0) -> float:
        r = ctypes.c_double()
        _check(self.ctx, lib.admm_get_rho(self.ctx, patient, ctypes.byref(r)))
        return r.value

    def z(self, patient: int = 0):
        z = np.zeros(self.n[patient])
        _check(self.ctx, lib.admm_get_z(self.ctx, patient, z.ctypes.data))
        return z

    def get_state(self, patient: int = 0):
        n, N = self.n[patient], self.num_scen[patient]
        z = np.zeros(n)
        y = np.zeros(N * n)
        d = np.zeros(N * n)
        sc = np.zeros(16)
        _check(self.ctx, lib.admm_get_state(self.ctx, patient, z.ctypes.data, y.ctypes.data, d.ctypes.data,
                                            sc.ctypes.data))
        return dict(z=z, y=y, d=d, scalars=sc)

    def set_state(self, state: dict, patient: int = 0):
        arrs = [np.ascontiguousarray(state[k], dtype=np.float64) for k in ("z", "y", "d", "scalars")]
        _check(self.ctx, lib.admm_set_state(self.ctx, patient, *[a.ctypes.data for a in arrs]))

    def trace(self, patient: int = 0, cap: int = 100000) -> List[dict]:
        buf = (InfoC * cap)()
        cnt = ctypes.c_int32()
        _check(self.ctx, lib.admm_get_trace(self.ctx, patient, buf, cap, ctypes.byref(cnt)))
        return [buf[i].as_dict() for i in range(cnt.value)]

    def tuning(self, patient: Optional[int] = None):
        """The sparse-pass configuration: of the context (patient 0's, and the
        summed tuned pass time), or of one patient."""
        t, u, a, f = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ms = ctypes.c_double()
        if patient is None:
            _check(self.ctx, lib.admm_get_tuning(self.ctx, ctypes.byref(t), ctypes.byref(u), ctypes.byref(a),
                                                 ctypes.byref(ms)))
            _check(self.ctx, lib.admm_get_format(self.ctx, ctypes.byref(f)))
        else:
            _check(self.ctx, lib.admm_get_pass_config(self.ctx, int(patient), ctypes.byref(t), ctypes.byref(u),
                                                      ctypes.byref(a), ctypes.byref(f), ctypes.byref(ms)))
        return dict(threads=t.value, unroll=u.value, lds_acc=a.value, pass_ms=ms.value,
                    format="sell" if f.value == 1 else "csr")

    def forward_config(self, patient: int = 0):
        """Workgroup size, row pipelining and tuned time (ms) of one patient's
        forward, objective and transpose products."""
        t, u, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(self.ctx, lib.admm_get_forward_config(self.ctx, int(patient), ctypes.byref(t), ctypes.byref(u),
                                                     ctypes.byref(ms)))
        return dict(threads=t.value, unroll=u.value, pass_ms=ms.value)

    def cg_counts(self, patient: int = 0):
        c = np.zeros(self.num_scen[patient], dtype=np.int64)
        _check(self.ctx, lib.admm_get_cg_counts(self.ctx, patient, c.ctypes.data))
        return c

    def sizes(self, patient: int = 0):
        n, m, N = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        nnz = ctypes.c_int64()
        _check(self.ctx, lib.admm_get_sizes(self.ctx, patient, ctypes.byref(n), ctypes.byref(m), ctypes.byref(N),
                                            ctypes.byref(nnz)))
        return dict(n=n.value, m=m.value, num_scen=N.value, nnz=nnz.value)

    def xupdate(self):
        """('cg' or 'dense', device ms of the last cached-inverse set-up)."""
        mode, ms = ctypes.c_int32(), ctypes.c_double()
        _check(self.ctx, lib.admm_get_xupdate(self.ctx, ctypes.byref(mode), ctypes.byref(ms)))
        return ("dense" if mode.value == 1 else "cg"), ms.value

    def time_pass(self, kind: str, reps: int = 20) -> float:
        """Average ms of one sparse pass over all scenarios: 'forward', 'transpose' or 'normal'."""
        k = {"forward": 0, "transpose": 1, "normal": 2}[kind]
        ms = ctypes.c_double()
        _check(self.ctx, lib.admm_time_pass(self.ctx, k, int(reps), ctypes.byref(ms)))
        return ms.value

    def enable_timing(self, on: bool = True):
        _check(self.ctx, lib.admm_enable_timing(self.ctx, 1 if on else 0))

    def timing(self):
        t, p = ctypes.c_double(), ctypes.c_double()
        c = ctypes.c_int32()
        _check(self.ctx, lib.admm_get_timing(self.ctx, ctypes.byref(t), ctypes.byref(p), ctypes.byref(c)))
        return dict(total_ms=t.value, pass_ms=p.value, pass_launches=c.value)


def _mlp_check(code: int):
    if code < 0:
        raise AdmmError(code, lib.mlp_last_error().decode(errors="replace"))
    return code


class Mlp:
    """The warm-start network of the library (training and inference on the GPU)."""

    def __init__(self, nin: int, hidden: int = 128, seed: int = 0, stream=None):
        st = None if stream is None else int(getattr(stream, "cuda_stream", stream))
        h = ctypes.c_void_p()
        _mlp_check(lib.mlp_create(int(nin), int(hidden), ctypes.c_uint64(seed), st, ctypes.byref(h)))
        self.h = h
        self.nin, self.hidden = int(nin), int(hidden)

    def close(self):
        if getattr(self, "h", None):
            lib.mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    @property
    def num_params(self) -> int:
        return int(lib.mlp_num_params(self.h))

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.num_params, dtype=np.float32)
        _mlp_check(lib.mlp_get_params(self.h, out.ctypes.data))
        return out

    def set_params(self, theta) -> None:
        t = np.ascontiguousarray(theta, dtype=np.float32)
        if t.shape[0] != self.num_params:
            raise ValueError("parameter count mismatch")
        _mlp_check(lib.mlp_set_params(self.h, t.ctypes.data))

    def forward(self, X, precision="fp32"):
        Xa = np.ascontiguousarray(X, dtype=np.float32)
        y = np.zeros(Xa.shape[0], dtype=np.float32)
        lr = ctypes.c_float()
        pr = PREC[precision] if isinstance(precision, str) else int(precision)
        _mlp_check(lib.mlp_forward(self.h, Xa.ctypes.data, Xa.shape[0], pr, y.ctypes.data, ctypes.byref(lr)))
        return y, lr.value

    def loss_grad(self, X, target, target_log_rho: float = 0.0, lam: float = 0.0, want_grad: bool = True):
        Xa = np.ascontiguousarray(X, dtype=np.float32)
        ta = np.ascontiguousarray(target, dtype=np.float32)
        loss = ctypes.c_double()
        g = np.zeros(self.num_params, dtype=np.float32) if want_grad else None
        _mlp_check(lib.mlp_loss_grad(self.h, Xa.ctypes.data, ta.ctypes.data, Xa.shape[0], float(target_log_rho),
                                     float(lam), ctypes.byref(loss), _ptr(g)))
        return loss.value, g

    def adam_step(self, lr: float = 1e-3, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        _mlp_check(lib.mlp_adam_step(self.h, float(lr), float(beta1), float(beta2), float(eps)))
