"""Input generator: determinism, CSR invariants, and the R-MAT distribution."""
import hashlib

import numpy as np
import pytest

import rmatgen


def digest(g):
    h = hashlib.sha256()
    for a in (g.off.astype(np.int64), g.dst, g.w if g.w is not None else np.zeros(0, np.uint32)):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def check_csr(g, symmetric=False):
    off = g.off.astype(np.int64)
    assert off[0] == 0 and off[-1] == g.m and np.all(np.diff(off) >= 0)
    assert g.dst.dtype == np.int32 and g.dst.size == g.m
    if g.m:
        assert g.dst.min() >= 0 and g.dst.max() < g.n
    srcs = np.repeat(np.arange(g.n), np.diff(off))
    assert not np.any(srcs == g.dst), "self-loop"
    key = srcs.astype(np.int64) * g.n + g.dst
    assert np.all(np.diff(key) > 0), "adjacency lists must be sorted and duplicate-free"
    if symmetric:
        rev = g.dst.astype(np.int64) * g.n + srcs
        assert np.array_equal(np.sort(rev), key)
    if g.w is not None:
        assert g.w.dtype == np.uint32 and g.w.min() >= 1 and g.w.max() <= 255


@pytest.mark.parametrize("directed", [True, False])
def test_same_seed_same_graph_any_thread_count(directed):
    a = rmatgen.rmat(13, 16, seed=42, directed=directed, weighted=True, threads=1)
    b = rmatgen.rmat(13, 16, seed=42, directed=directed, weighted=True, threads=7)
    assert digest(a) == digest(b)
    c = rmatgen.rmat(13, 16, seed=43, directed=directed, weighted=True)
    assert digest(a) != digest(c)
    check_csr(a, symmetric=not directed)


def test_int32_offsets_match_int64():
    a = rmatgen.rmat(12, 8, seed=1, offset_dtype=np.int64)
    b = rmatgen.rmat(12, 8, seed=1, offset_dtype=np.int32)
    assert b.off.dtype == np.int32 and np.array_equal(a.off, b.off) and np.array_equal(a.dst, b.dst)


def test_quadrant_frequencies_follow_abcd():
    # per level, (src bit, dst bit) = (0,0),(0,1),(1,0),(1,1) with probabilities a, b, c, d
    s, d = rmatgen.rmat_samples(10, 0, 400_000)
    counts = np.zeros(4)
    for lvl in range(10):
        sb = (s >> lvl) & 1
        db = (d >> lvl) & 1
        counts += np.bincount(sb * 2 + db, minlength=4)
    freq = counts / counts.sum()
    assert np.allclose(freq, [0.57, 0.19, 0.19, 0.05], atol=2e-3)


def test_weights_uniform_on_1_255():
    g = rmatgen.rmat(14, 16, weighted=True)
    hist = np.bincount(g.w, minlength=256)[1:]
    assert hist.min() > 0.8 * g.m / 255 and hist.max() < 1.2 * g.m / 255


def test_from_edges_cleans_and_raw_keeps():
    g = rmatgen.from_edges(4, [0, 0, 0, 1, 2, 3], [1, 1, 0, 2, 2, 0])
    assert g.off.tolist() == [0, 1, 2, 2, 3] and g.dst.tolist() == [1, 2, 0]
    r = rmatgen.raw_csr(4, [0, 0, 0, 1, 2, 3], [1, 1, 0, 2, 2, 0])
    assert r.off.tolist() == [0, 3, 4, 5, 6] and r.dst.tolist() == [1, 1, 0, 2, 2, 0]


def test_workload_shapes_small_scale():
    g = rmatgen.workload("pr-s16", scale=10)
    assert g.n == 1024 and g.off.dtype == np.int32 and g.w is None
    check_csr(g)
    g = rmatgen.workload("cc-s22", scale=10)
    check_csr(g, symmetric=True)
    g = rmatgen.workload("sssp-s26", scale=10)
    assert g.off.dtype == np.int64 and g.w is not None
    check_csr(g)
