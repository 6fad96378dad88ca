"""The C-ABI library on the host: it loads, exports every function the header
declares, and reports malformed input with the documented codes before any
device work (no GPU needed)."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "admmbb.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = _declared_functions()
    for required in ("admm_setup", "admm_setup_batch", "admm_warm_start", "admm_iterate", "admm_solve",
                     "pgd_solve", "admm_objective", "admm_kkt", "admm_get_state", "admm_set_state",
                     "admm_last_error", "admm_destroy", "admm_spot_features", "mlp_forward", "mlp_loss_grad",
                     "mlp_adam_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2304_14568_amd as A
    missing = [n for n in _declared_functions() if not hasattr(A.lib, n)]
    assert not missing, missing
    assert set(A.EXPORTS) <= set(_declared_functions())


def _tiny():
    return synth.make_tiny(0)


def _codes():
    import paper_2304_14568_amd as A
    return A


def _mutated(**changes):
    P = _tiny()
    A0 = P.A[0]
    csr = synth.Csr(row_ptr=A0.row_ptr.copy(), col=A0.col.copy(), val=A0.val.copy())
    for k, v in changes.items():
        v(P, csr)
    P.A = [csr] + list(P.A[1:])
    return P


def _first_nonempty_row(csr):
    return int(np.nonzero(np.diff(csr.row_ptr) >= 2)[0][0])


@pytest.mark.parametrize("case,code", [
    ("ok", 0),
    ("negative_value", -3),
    ("nan_value", -4),
    ("column_out_of_range", -2),
    ("columns_not_increasing", -2),
    ("row_ptr_decreasing", -2),
    ("negative_weight", -3),
    ("negative_prescription", -3),
    ("infinite_prescription", -4),
    ("struct_id_out_of_range", -1),
    ("lb_above_ub", -1),
    ("negative_probability", -3),
])
def test_validation_codes(case, code):
    A = _codes()

    def neg(P, c):
        c.val[0] = -1.0

    def nan(P, c):
        c.val[1] = np.nan

    def colr(P, c):
        r = _first_nonempty_row(c)
        c.col[c.row_ptr[r + 1] - 1] = P.n

    def colinc(P, c):
        r = _first_nonempty_row(c)
        b = c.row_ptr[r]
        c.col[b], c.col[b + 1] = c.col[b + 1], c.col[b]

    def rowdec(P, c):
        r = _first_nonempty_row(c)
        c.row_ptr[r + 1] = c.row_ptr[r + 2] + 1  # row r + 1 ends before it starts

    def negw(P, c):
        P.struct_weight = np.array(P.struct_weight, dtype=np.float64)
        P.struct_weight[0] = -0.5

    def negp(P, c):
        P.presc = np.array(P.presc, dtype=np.float64)
        P.presc[3] = -1.0

    def infp(P, c):
        P.presc = np.array(P.presc, dtype=np.float64)
        P.presc[3] = np.inf

    def sid(P, c):
        P.struct_id = np.array(P.struct_id, dtype=np.uint8)
        P.struct_id[0] = len(P.struct_weight)

    def lbub(P, c):
        P.lb = np.array(P.lb, dtype=np.float64)
        P.lb[0] = float(P.ub[0]) + 1.0

    def negprob(P, c):
        P.prob = np.array(P.prob, dtype=np.float64)
        P.prob[0] = -1.0

    muts = dict(ok=lambda P, c: None, negative_value=neg, nan_value=nan, column_out_of_range=colr,
                columns_not_increasing=colinc, row_ptr_decreasing=rowdec, negative_weight=negw,
                negative_prescription=negp, infinite_prescription=infp, struct_id_out_of_range=sid,
                lb_above_ub=lbub, negative_probability=negprob)
    P = _mutated(m=muts[case])
    got = A.validate(P)
    assert got == code, (case, got, A.last_setup_error())
    if code != 0:
        assert A.last_setup_error()


def test_bad_options_rejected_before_device_work():
    A = _codes()
    P = _tiny()
    for kw in (dict(cg_max=0), dict(cg_max=65), dict(z_mode=2), dict(lds_acc=3), dict(pass_threads=128),
               dict(pass_unroll=3), dict(max_iter=-1), dict(check_every=0), dict(precision=7),
               dict(xupdate=2), dict(format=2), dict(deterministic=2), dict(deterministic=1, lds_acc=1),
               dict(dense_launches=5)):
        with pytest.raises(A.AdmmError) as e:
            A.Solver(P, **kw)
        assert e.value.code == -1, kw


def test_setup_without_device_reports_hip_error():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a device is present")
    A = _codes()
    with pytest.raises(A.AdmmError) as e:
        A.Solver(_tiny())
    assert e.value.code == -6
    with pytest.raises(A.AdmmError) as e:
        A.Mlp(4, 8)
    assert e.value.code == -6


def test_default_options_documented_values():
    A = _codes()
    o = A.default_options()
    assert o.obj_rel_tol == 1e-5 and o.eps_abs == 1e-6 and o.eps_rel == 1e-6
    assert o.bb == 1 and o.z_mode == 0 and o.bb_clamp == 0.0
    assert o.cg_max == 8 and o.max_iter == 1000
    assert o.xupdate == -1  # automatic choice between the dense and the CG x-update


def test_too_many_spots_for_the_sparse_pass_rejected():
    import paper_2304_14568_amd as A
    from tests._helpers import problem_from_dense
    n = 13700
    D = np.zeros((2, n))
    D[0, 0] = 1.0
    D[1, 1] = 1.0
    P = problem_from_dense([D], w=[1.0, 1.0], p=[1.0, 1.0])
    with pytest.raises(A.AdmmError) as e:
        A.Solver(P)
    assert e.value.code == -1 and "13 600" in str(e.value)


def test_stream_probe_rejects_bad_arguments_before_device_work():
    import paper_2304_14568_amd as A
    gbs = ctypes.c_double()
    assert A.lib.admm_stream_probe(0, 1, ctypes.byref(gbs)) == A.E_ARG          # below 1 MiB
    assert A.lib.admm_stream_probe(1 << 30, 0, ctypes.byref(gbs)) == A.E_ARG    # no passes
    assert A.lib.admm_stream_probe(17 << 30, 1, ctypes.byref(gbs)) == A.E_ARG   # above 16 GiB
    assert A.lib.admm_stream_probe(1 << 30, 1, None) == A.E_ARG


def test_memory_kind_checked_on_the_host():
    """An unknown mem_kind is refused, and host-only validation refuses a
    problem whose CSR arrays are device memory (it cannot read them)."""
    A = _codes()
    P = _tiny()
    for kind in (1, 7):
        h = A._ProblemHold(P)
        h.c.mem_kind = kind
        assert A.lib.admm_validate(h.c) == -1
        assert "mem_kind" in A.last_setup_error() or "device" in A.last_setup_error()
