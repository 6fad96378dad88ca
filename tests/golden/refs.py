"""Read the stored oracle results of tests/golden (JSON only; imports nothing else).

The files are written by make_references.py from the generator and the oracle;
readers that must not touch the oracle (the benchmark, the experiments) use
this module."""
from __future__ import annotations

import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def load(name: str):
    """Return (record, x_star) or (None, None) when no stored file exists."""
    path = os.path.join(HERE, f"{name}.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as fh:
        rec = json.load(fh)
    x = np.zeros(rec["n"])
    for k, v in rec["x_star_nonzero"].items():
        x[int(k)] = v
    return rec, x
