"""Batched CC / SSSP over many graphs in one run (GPU): every member's
result must equal the oracle's and the member's own plain run, bit for bit."""
import numpy as np
import pytest

import oracle
import rmatgen

pytestmark = pytest.mark.gpu


def mixed_members(seed, count, lo=5, hi=12):
    rng = np.random.default_rng(seed)
    csrs, queries = [], []
    for i in range(count):
        sc, ef = int(rng.integers(lo, hi + 1)), int(rng.integers(2, 17))
        if rng.random() < 0.5:
            c = rmatgen.rmat(sc, ef, seed=seed * 1000 + i, directed=False,
                             offset_dtype=np.int32 if i % 3 else np.int64)
            queries.append(("cc", 0))
        else:
            c = rmatgen.rmat(sc, ef, seed=seed * 1000 + i, weighted=bool(rng.random() < 0.7))
            queries.append(("sssp", int(rng.integers(0, c.n))))
        csrs.append(c)
    # edge cases: one vertex, no edges, SSSP from an isolated vertex
    csrs.append(rmatgen.raw_csr(1, [], []))
    queries.append(("sssp", 0))
    csrs.append(rmatgen.raw_csr(7, [], []))
    queries.append(("cc", 0))
    iso = rmatgen.raw_csr(5, [0, 1, 2], [1, 2, 3], [4, 5, 6])
    csrs.append(iso)
    queries.append(("sssp", 4))
    return csrs, queries


@pytest.mark.parametrize("sched", ["auto", "edge", "pull", "vertex"])
@pytest.mark.parametrize("relabel", [True, False])
def test_batch_members_match_oracle(device, sched, relabel):
    from paper_2010_01542_amd import Batch
    print(f"case batch 40 members schedule={sched} relabel={relabel}", flush=True)
    csrs, queries = mixed_members(5, 40)
    b = Batch(csrs, queries, relabel=relabel)
    out, st = b.run(schedule=sched, stats=True)
    for c, (prog, src), got in zip(csrs, queries, b.split(out)):
        ref = oracle.run(prog, c.n, c.off, c.dst, c.w if prog == "sssp" else None, source=src)
        assert np.array_equal(got, ref.values), (prog, c.n, c.m)
    assert st.supersteps >= 1


def test_batch_equals_solo_runs(device):
    from paper_2010_01542_amd import Batch, Graph
    csrs, queries = mixed_members(9, 24, lo=8, hi=13)
    b = Batch(csrs, queries)
    out, st = b.run(stats=True)
    edges = 0
    for c, (prog, src), got in zip(csrs, queries, b.split(out)):
        solo, sst = Graph.from_csr(c).run(prog, source=src, stats=True)
        assert np.array_equal(got, solo.cpu().numpy().view(np.uint32))
        edges += sst.edges_relaxed
    # the union's per-superstep messages are the members' messages, superstep by superstep
    assert st.edges_relaxed == edges


def test_batch_rejects_bad_queries(device):
    from paper_2010_01542_amd import Batch, VcError
    c = rmatgen.path(4)
    with pytest.raises(VcError):
        Batch([c], [("pagerank", 0)])
    with pytest.raises(VcError):
        Batch([c], [("sssp", 4)])
