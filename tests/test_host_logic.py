"""Host-side logic of the package that needs no GPU: warm-start features,
histogram sizing, the benchmark's kernel-source key, and the stored oracle
references against the generator."""
from __future__ import annotations

import importlib.util
import os

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_geometric_features_and_voxel_classes():
    from paper_2304_14568_amd import warmstart as W
    P = synth.hn_small(3)
    X = W.geometric_features(P)
    assert X.shape == (P.n, W.GEOM_FEATURES) and np.all(np.isfinite(X))
    assert np.all((X[:, 0] >= 0) & (X[:, 0] <= 1))          # layer position within its beam
    assert np.allclose(X[:, 5:8].sum(axis=1), 1.0)           # beam one-hot
    assert np.allclose(X[:, 4], np.hypot(X[:, 2], X[:, 3]), atol=1e-6)
    vc = W.voxel_class(P)
    names = P.meta["struct_names"]
    for g, nm in enumerate(names):
        sel = np.asarray(P.struct_id) == g
        want = 1 if nm.startswith("target") else 2 if nm.startswith("oar") else 0
        assert np.all(vc[sel] == want)


def test_histogram_size_fits_lds():
    from paper_2304_14568_amd.clinical import max_bins
    for G in (1, 7, 64, 256):
        nb = max_bins(G)
        assert 12 * G + 4 * G * nb <= 65536 < 12 * G + 4 * G * (nb + 1)


def test_bench_kernel_source_key():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    src = os.path.join(ROOT, "paper_2304_14568_amd", "csrc", "factor.hip")
    key = bench.kernel_source_hash(src, "__global__ __launch_bounds__(256) void k_xsym(")
    assert len(key) == 16
    assert bench.kernel_source_hash(src, "no such kernel(") == ""


@pytest.mark.slow
def test_stored_references_match_the_generator():
    """Every stored oracle minimum of the scenario-count study still describes
    the instance the generator produces (content digest)."""
    from tests.golden.refs import load
    P = synth.hn_full(0)
    for N in (1, 5, 12):
        rec, x = load(f"hn_full_s0_n{N}")
        assert rec is not None and rec["digest"] == P.subset(list(range(N))).digest()
        assert rec["kkt"] <= 1e-12 and x.shape == (P.n,)
    rec, _ = load("hn_full_s0")
    assert rec["digest"] == P.digest()
    # more scenarios, larger minimum
    fs = [load(f"hn_full_s0_n{N}")[0]["f_star"] for N in range(1, 13)] + [rec["f_star"]]
    assert all(a < b for a, b in zip(fs, fs[1:]))


def test_gram_pair_index_multiply_shift_is_exact():
    """The tile Gram kernel splits a pair index p of an nI x nJ block of
    products as a = p / nJ, computed as (p * (2^19 // nJ + 1)) >> 19 in 32-bit
    arithmetic.  A row's segment in one 64-column block holds at most 64
    nonzeros plus 3 entries of padding, so nJ <= 67 and p < 67 * 67; the
    formula must be exact on that whole range and must not overflow."""
    for nJ in range(1, 68):
        m = (1 << 19) // nJ + 1
        p = np.arange(67 * 67, dtype=np.uint64)
        assert int(p.max()) * m < 2 ** 32
        a = ((p * np.uint64(m)) & np.uint64(0xFFFFFFFF)) >> np.uint64(19)
        assert np.array_equal(a, p // np.uint64(nJ))
