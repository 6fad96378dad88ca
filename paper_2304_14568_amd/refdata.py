"""Reader of stored reference minima (JSON records with f*, the nonzero entries
of x*, kappa(H) and the generator's content digest of the workload).

The records are written once by a script that runs the float64 reference
solver; this module only parses them, so the benchmark and the experiments can
report gaps to f* without running that solver.  Directory: the `directory`
argument, else the environment variable ADMMBB_REFS, else the repository's
tests/golden."""
from __future__ import annotations

import json
import os

import numpy as np

_DEFAULT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden")


def ref_dir(directory: str | None = None) -> str:
    return directory or os.environ.get("ADMMBB_REFS") or _DEFAULT


def load(name: str, directory: str | None = None):
    """(record, x_star) of `name`.json, or (None, None) when there is no such file."""
    path = os.path.join(ref_dir(directory), f"{name}.json")
    if not os.path.exists(path):
        return None, None
    with open(path) as fh:
        rec = json.load(fh)
    x = np.zeros(rec["n"])
    for k, v in rec["x_star_nonzero"].items():
        x[int(k)] = v
    return rec, x


def fstar(name: str, digest: str, directory: str | None = None):
    """f* of `name` when the stored record matches the workload's digest, else None."""
    rec, _ = load(name, directory)
    return rec["f_star"] if (rec is not None and rec["digest"] == digest) else None
