"""Error paths of the library on the GPU: documented status codes, no state
change on rejected calls."""
from __future__ import annotations

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    return synth.make_tiny(3)


@pytest.mark.parametrize("xupdate", ["cg", "dense"])
def test_iteration_limit_reports_max_iter(P, xupdate):
    import paper_2304_14568_amd as A
    with A.Solver(P, max_iter=3, xupdate=xupdate) as S:
        zs, info, st = S.solve()
        assert st == 1 and info[0]["iter"] == 3 and info[0]["status"] == 1
        assert np.all(np.isfinite(zs[0]))


def test_rejected_calls_leave_the_state(P):
    import paper_2304_14568_amd as A
    with A.Solver(P) as S:
        S.iterate(4)
        before = S.get_state()
        bad = {k: v.copy() for k, v in before.items()}
        bad["y"][0] = np.nan
        with pytest.raises(A.AdmmError) as e:
            S.set_state(bad)
        assert e.value.code == -4
        after = S.get_state()
        for k in ("z", "y", "d", "scalars"):
            assert np.array_equal(before[k], after[k])
        with pytest.raises(A.AdmmError) as e:
            S.objective(np.zeros(P.n), patient=1)
        assert e.value.code == -1
        with pytest.raises(A.AdmmError) as e:
            S.dose_stats(np.zeros(P.n), np.full(P.m, 9, dtype=np.uint8), 3, 16, 1.0)
        assert e.value.code == -1
        with pytest.raises(A.AdmmError) as e:
            S.dose_stats(np.zeros(P.n), np.zeros(P.m, dtype=np.uint8), 256, 4096, 1.0)
        assert e.value.code == -1
        with pytest.raises(A.AdmmError) as e:
            S.spot_features(np.full(P.m, 3, dtype=np.uint8))
        assert e.value.code == -1


def test_dense_request_beyond_its_limit_is_refused():
    import paper_2304_14568_amd as A
    # n > 8128: the dense x-update must refuse (the CG one accepts the same problem)
    P = synth.make_hn(seed=7, grid=(72, 72, 48), body_semi_vox=(30, 24, 18), target_size=1.1, num_layers=16,
                      spot_spacing=2.5, num_scen=1)
    assert 8128 < P.n <= 13000
    with pytest.raises(A.AdmmError) as e:
        A.Solver(P, xupdate="dense")
    assert e.value.code == -1
    with A.Solver(P, xupdate="auto") as S:
        assert S.xupdate()[0] == "cg"
