"""Captured (HIP graph) superstep loops and the autotuner (GPU).

A captured run must give the oracle's values and the oracle's per-superstep
frontier sizes (recorded on the device); replays are interleaved with eager
work and re-captures, and every replay is checked.  Captured CC / SSSP loops
pick each superstep's form on the device (edge-balanced push below the
dense threshold, the pull or, from 2^20 vertices, the blocked form above
it): the forms they record must be the ones the host loop picks, and every
form alone (explicit schedules) must give the same results."""
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


@pytest.mark.parametrize("sched", ["edge", "pull", "vertex"])
def test_captured_loop_with_fixed_forms(device, sched):
    """Explicit schedules fix the captured loop's form: pushed (edge-balanced,
    for "edge" and "vertex") or pulled in every superstep."""
    from paper_2010_01542_amd import vc
    cap = vc.OPT_GRAPH_CAPTURE
    d = rmatgen.rmat(14, 12, seed=31, weighted=True)
    u = rmatgen.rmat(14, 12, seed=32, directed=False)
    gd, gu = make(d), make(u, symmetric=True)
    print(f"case captured loop schedule={sched}", flush=True)
    want = vc.SCHED_PULL if sched == "pull" else vc.SCHED_EDGE
    for g, c, prog in ((gd, d, "sssp"), (gu, u, "cc")):
        for _ in range(2):
            _, st, _ = check_min(c, g, prog, source=3, schedule=sched, options=cap)
            used = [x for x in st.schedule.tolist()[1:] if x]
            assert used and set(used) == {want}, st.schedule.tolist()


@pytest.fixture(scope="module")
def big_pair():
    """Graphs of 2^20 vertices, where AUTO's dense supersteps take the blocked form."""
    d = rmatgen.rmat(20, 6, seed=33, weighted=True)
    u = rmatgen.rmat(20, 3, seed=34, directed=False)
    return d, u


def test_captured_loop_switches_forms_on_the_device(device, big_pair):
    """AUTO in a captured loop on a 2^20-vertex graph: the device picks the
    blocked form for dense supersteps and the push for the rest, exactly as
    the host loop does, with the oracle's values and frontier sizes."""
    from paper_2010_01542_amd import vc
    cap = vc.OPT_GRAPH_CAPTURE
    d, u = big_pair
    gd, gu = make(d), make(u, symmetric=True)
    for g, c, prog in ((gd, d, "sssp"), (gu, u, "cc")):
        print(f"case captured loop 2^20 {prog}", flush=True)
        _, host, _ = check_min(c, g, prog, source=0)
        # the host loop pushes tiny frontiers vertex-per-thread, the captured one edge-balanced
        want = [vc.SCHED_EDGE if x == vc.SCHED_VERTEX else x for x in host.schedule.tolist()]
        for _ in range(2):
            _, st, _ = check_min(c, g, prog, source=0, options=cap)
            assert st.schedule.tolist()[1:] == want[1:], (st.schedule.tolist(), host.schedule.tolist())
        used = set(st.schedule.tolist()[1:])
        assert vc.SCHED_BLOCKED in used and vc.SCHED_EDGE in used, st.schedule.tolist()
        _, st, _ = check_min(c, g, prog, source=0, schedule="blocked", options=cap)
        assert set(x for x in st.schedule.tolist()[1:] if x) == {vc.SCHED_BLOCKED}
