"""Small helpers shared by the tests (problem construction from dense arrays)."""
from __future__ import annotations

import dataclasses
import json
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name: str) -> dict:
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def csr_from_dense(D) -> synth.Csr:
    D = np.asarray(D, dtype=np.float32)
    rows, cols = np.nonzero(D)
    row_ptr = np.zeros(D.shape[0] + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return synth.Csr(row_ptr=row_ptr, col=cols.astype(np.int32), val=D[rows, cols].astype(np.float32))


def problem_from_dense(As, w, p, lb=None, ub=None, c=None) -> synth.Problem:
    """Build a Problem with one structure per voxel (so any w is representable)."""
    As = [np.asarray(a, dtype=np.float64) for a in As]
    m, n = As[0].shape
    w = np.asarray(w, dtype=np.float64)
    return synth.Problem(
        m=m, n=n, A=[csr_from_dense(a) for a in As],
        prob=np.ones(len(As)) if c is None else np.asarray(c, dtype=np.float64),
        struct_id=np.arange(m, dtype=np.uint8) if m < 256 else np.zeros(m, dtype=np.uint8),
        struct_weight=w if m < 256 else w[:1],
        presc=np.asarray(p, dtype=np.float64),
        lb=np.zeros(n) if lb is None else np.asarray(lb, dtype=np.float64),
        ub=np.full(n, np.inf) if ub is None else np.asarray(ub, dtype=np.float64),
        name="dense")


def with_presc(P: synth.Problem, presc) -> synth.Problem:
    return dataclasses.replace(P, presc=np.asarray(presc, dtype=np.float64))


def with_weights(P: synth.Problem, struct_weight) -> synth.Problem:
    return dataclasses.replace(P, struct_weight=np.asarray(struct_weight, dtype=np.float64))


def duplicate_scenario(P: synth.Problem, s: int) -> synth.Problem:
    A = list(P.A) + [P.A[s]]
    return dataclasses.replace(P, A=A, prob=np.concatenate([P.prob, [P.prob[s]]]))


def scaled_prob(P: synth.Problem, s: int, factor: float) -> synth.Problem:
    c = P.prob.copy()
    c[s] = c[s] * factor
    return dataclasses.replace(P, prob=c)
