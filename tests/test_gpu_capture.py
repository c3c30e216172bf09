"""Captured (HIP graph) superstep loops and the autotuner (GPU).

A captured run must give the oracle's values and the oracle's per-superstep
frontier sizes (recorded on the device); replays are interleaved with eager
work and re-captures, and every replay is checked."""
import numpy as np
import pytest

import oracle
import rmatgen
from gpu_util import check_min, check_rank, run_gpu

pytestmark = pytest.mark.gpu


def make(csr, **kw):
    from paper_2010_01542_amd import Graph
    return Graph.from_csr(csr, **kw)


@pytest.mark.parametrize("relabel", [True, False])
def test_captured_min_programs_match_oracle(device, relabel):
    from paper_2010_01542_amd import vc
    cap = vc.OPT_GRAPH_CAPTURE
    d = rmatgen.rmat(13, 16, seed=17, weighted=True)
    u = rmatgen.rmat(13, 16, seed=18, directed=False)
    gd, gu = make(d, relabel=relabel), make(u, relabel=relabel)
    for src in (0, 5, d.n - 1, 0):  # replays of the cached graph, new sources
        check_min(d, gd, "sssp", source=src, options=cap)
        check_rank(d, gd, "pagerank", T=3)  # eager work between replays
    for _ in range(3):
        check_min(u, gu, "cc", options=cap)
    for c in (rmatgen.path(40), rmatgen.cliques([5, 1, 9], isolated=4), rmatgen.raw_csr(1, [], [])):
        check_min(c, make(c, relabel=relabel), "cc", options=cap)
        check_min(c, make(c, relabel=relabel), "sssp", source=0, options=cap)


def test_captured_pagerank_and_ppr(device):
    from paper_2010_01542_amd import vc
    cap = vc.OPT_GRAPH_CAPTURE
    d = rmatgen.rmat(12, 16, seed=3)
    g = make(d)
    for T in (10, 10, 4, 10):  # cached, re-captured, cached again
        check_rank(d, g, "pagerank", T=T, options=cap)
    check_rank(d, g, "ppr", T=8, source=3, options=cap)
    check_rank(d, g, "pagerank", T=10, schedule="edge", options=cap)
    a = run_gpu(g, "pagerank", T=10, options=cap)[0]
    b = run_gpu(g, "pagerank", T=10)[0]
    assert np.array_equal(a, b)
    g2 = make(d, relabel=False)
    check_rank(d, g2, "pagerank", T=6, options=cap)


def test_captured_cap_reports_not_converged(device):
    from paper_2010_01542_amd import VcError, vc
    g = make(rmatgen.path(60))
    with pytest.raises(VcError) as e:
        g.run("cc", max_supersteps=20, options=vc.OPT_GRAPH_CAPTURE)
    assert e.value.status == vc.ERR_NOT_CONVERGED


def test_captured_batch(device):
    from paper_2010_01542_amd import Batch, vc
    from test_gpu_batch import mixed_members
    csrs, queries = mixed_members(12, 20)
    b = Batch(csrs, queries)
    for _ in range(2):
        out, _ = b.run(options=vc.OPT_GRAPH_CAPTURE)
        for c, (prog, src), got in zip(csrs, queries, b.split(out)):
            ref = oracle.run(prog, c.n, c.off, c.dst, c.w if prog == "sssp" else None, source=src)
            assert np.array_equal(got, ref.values)


def test_autotune_keeps_results_exact(device):
    from paper_2010_01542_amd import Batch
    d = rmatgen.rmat(13, 16, seed=23, weighted=True)
    g = make(d)
    best = g.autotune("sssp", source=0)
    assert best["tile"] in (1024, 2048, 4096)
    check_min(d, g, "sssp", source=0)  # AUTO now runs the tuned setting
    best = g.autotune("pagerank", T=10)
    assert best["schedule"] in ("pull", "edge", "blocked")
    check_rank(d, g, "pagerank", T=10)
    from test_gpu_batch import mixed_members
    csrs, queries = mixed_members(13, 12)
    b = Batch(csrs, queries)
    b.autotune()
    out, _ = b.run()
    for c, (prog, src), got in zip(csrs, queries, b.split(out)):
        ref = oracle.run(prog, c.n, c.off, c.dst, c.w if prog == "sssp" else None, source=src)
        assert np.array_equal(got, ref.values)
