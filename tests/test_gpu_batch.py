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


def union_stats(refs):
    """Per-superstep senders and messages of the union: the members run in
    lockstep supersteps, so the union's counts are the members' sums, each
    member contributing zeros once it has quiesced."""
    steps = max(r.supersteps for r in refs)
    senders, messages = np.zeros(steps, np.int64), np.zeros(steps, np.int64)
    for r in refs:
        senders[: r.supersteps] += r.senders
        messages[: r.supersteps] += r.messages
    return steps, senders.tolist(), messages.tolist()


@pytest.fixture(scope="module", params=[False, True], ids=["byte-weights", "wide-weights"])
def big_union(request):
    """A union of more than 2^20 vertices, the size at which AUTO takes the
    blocked form for dense supersteps: 48 members of scales 14..16 (edge
    factor 8..32), symmetrised CC and weighted SSSP in [1, 255] (the
    benchmark's batch; the blocked layout then keeps one-byte slot weights)
    or with some members' weights beyond a byte (four-byte slot weights),
    plus an edgeless member and a lone vertex."""
    wide = request.param
    rng = np.random.default_rng(2024)
    csrs, queries = [], []
    for i in range(48):
        sc, ef = int(rng.integers(14, 17)), int(rng.integers(8, 33))
        if i % 2 == 0:
            csrs.append(rmatgen.rmat(sc, ef, seed=7000 + i, directed=False))
            queries.append(("cc", 0))
        else:
            c = rmatgen.rmat(sc, ef, seed=7000 + i, weighted=True)
            if wide and i % 6 == 1:
                c = rmatgen.Csr(c.n, c.m, c.off, c.dst, (c.w.astype(np.uint32) * 997).astype(np.uint32))
            csrs.append(c)
            queries.append(("sssp", int(rng.integers(0, c.n))))
    csrs.append(rmatgen.raw_csr(300, [], []))
    queries.append(("cc", 0))
    csrs.append(rmatgen.raw_csr(1, [], []))
    queries.append(("sssp", 0))
    refs = [oracle.run(p, c.n, c.off, c.dst, c.w if p == "sssp" else None, source=s)
            for c, (p, s) in zip(csrs, queries)]
    return csrs, queries, refs


@pytest.mark.parametrize("sched", ["blocked", "auto", "auto-captured"])
def test_large_union_takes_blocked_form_bit_exact(device, big_union, sched):
    """The union at the size where AUTO takes the blocked form, in the host
    loop and in the captured loop (whose forms are picked on the device)."""
    from paper_2010_01542_amd import Batch, vc
    csrs, queries, refs = big_union
    n = sum(c.n for c in csrs)
    assert n >= 1 << 20
    print(f"case batch union n={n} m={sum(c.m for c in csrs)} schedule={sched}", flush=True)
    b = Batch(csrs, queries)
    opts = vc.OPT_GRAPH_CAPTURE if sched.endswith("captured") else 0
    out, st = b.run(schedule=sched.split("-")[0], options=opts, stats=True)
    if opts:  # a second replay of the cached graph
        out, st = b.run(schedule="auto", options=opts, stats=True)
    for i, (c, (prog, src), got, ref) in enumerate(zip(csrs, queries, b.split(out), refs)):
        assert np.array_equal(got, ref.values), (i, prog, c.n, c.m, int((got != ref.values).sum()))
    steps, senders, messages = union_stats(refs)
    assert st.supersteps == steps
    assert st.frontier.tolist() == senders
    assert st.edges.tolist() == messages
    assert vc.SCHED_BLOCKED in st.schedule.tolist(), st.schedule.tolist()
