"""Write stored oracle results for the workloads too large to solve inside a test.

Calls only the generator (synth) and the oracle: the exact minimiser of the
box-constrained problem of Sec. 2.1 by the oracle's projected-Newton active-set
polish (KKT residual <= 1e-12), recorded with the generator's content digest so
a consumer can tell whether it still describes the same generated instance.

Usage:  python tests/golden/make_references.py [name ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import exact, wls  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

WORKLOADS = {
    "hn_full_s0": lambda: synth.hn_full(0),
}
# the same patient with its first N scenarios (scenario-count scaling, Sec. 3.3)
for _n in range(1, 13):
    WORKLOADS[f"hn_full_s0_n{_n}"] = (lambda n: (lambda: synth.hn_full(0).subset(list(range(n)))))(_n)
# the two smallest patients of the multi-patient batch recipe (seed 10), with
# their 64-scenario shift lattice
for _k in (2, 1):
    WORKLOADS[f"batch_s10_p{_k}"] = (lambda k: (lambda: synth.batch_patient(k, num=8, scen=64, seed=10)))(_k)


def make(name: str) -> dict:
    t0 = time.time()
    P = WORKLOADS[name]()
    W = wls.from_problem(P)
    H, g0, const = wls.quadratic_form(W)
    x, info = exact.active_set(W, H=H, g0=g0)
    f = wls.objective(W, x)
    ev = np.linalg.eigvalsh(H)
    nz = np.nonzero(x)[0]
    rec = {
        "_source": "oracle active-set minimiser of the robust WLS problem (Sec. 2.1) on a synth workload",
        "workload": name,
        "digest": P.digest(),
        "m": P.m, "n": P.n, "num_scen": P.num_scen, "nnz": P.nnz,
        "f_star": f,
        "kkt": info["kkt"],
        "cond_H": float(ev[-1] / ev[0]),
        "x_star_nonzero": {str(int(j)): float(x[j]) for j in nz},
        "seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    return rec


from tests.golden.refs import load  # noqa: E402,F401  (re-exported for the tests)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(WORKLOADS)):
        r = make(nm)
        print(nm, r["digest"], r["f_star"], r["kkt"], f"{r['seconds']:.1f}s")
