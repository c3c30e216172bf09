"""Pins of the CPU oracle against results fixed by mathematics, not by itself.

Each program of the oracle (paper, Section VI-C benchmarks run under the
Section I superstep model) is checked against an independent route to the
same result:

* hash-min CC   -> minimum vertex id of each connected component, from
                   scipy's connected_components and from a union-find written
                   here; exhaustive over all 1,024 undirected graphs on 5
                   vertices; closed forms for paths, cliques, isolated vertices.
* SSSP          -> Dijkstra (scipy, and a heap version written here), BFS
                   levels for unit weights; exhaustive over all 4,096 loop-free
                   digraphs on 4 vertices with seeded weights; prefix sums on a
                   weighted path.
* PageRank/PPR  -> exact rational arithmetic (fractions.Fraction) on tiny
                   graphs; the matrix-power closed form
                   r(T) = sum_{k<T} (d P^T)^k t + (d P^T)^T r(0);
                   closed forms on cycles, complete digraphs and stars; the
                   dangling-mass invariant.
* Per-superstep frontier sizes -> hop-bounded Bellman-Ford / label
                   propagation in dense matrix form, BFS level sizes, and the
                   path closed form N - s.
"""
import heapq
import itertools
from fractions import Fraction

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import breadth_first_order, connected_components, dijkstra, shortest_path

import oracle
import rmatgen

U = oracle.UNREACHED
D = 0.85


# ----------------------------------------------------------------------------- independent references

def min_id_components(n, src, dst):
    """Minimum vertex id of each weakly connected component (scipy)."""
    if n == 0:
        return np.zeros(0, np.uint32)
    a = csr_matrix((np.ones(len(src)), (np.asarray(src), np.asarray(dst))), shape=(n, n))
    _, lab = connected_components(a, directed=False)
    mins = np.full(lab.max() + 1, n, dtype=np.int64)
    np.minimum.at(mins, lab, np.arange(n))
    return mins[lab].astype(np.uint32)


def union_find_min(n, edges):
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for u, v in edges:
        ru, rv = find(u), find(v)
        if ru != rv:
            parent[max(ru, rv)] = min(ru, rv)
    return np.array([find(v) for v in range(n)], dtype=np.uint32)


def dijkstra_heap(n, arcs, src):
    """Textbook Dijkstra with a binary heap; arcs = [(u, v, w)]."""
    adj = [[] for _ in range(n)]
    for u, v, w in arcs:
        adj[u].append((v, w))
    dist = [None] * n
    dist[src] = 0
    heap = [(0, src)]
    done = [False] * n
    while heap:
        du, u = heapq.heappop(heap)
        if done[u]:
            continue
        done[u] = True
        for v, w in adj[u]:
            nd = du + w
            if dist[v] is None or nd < dist[v]:
                dist[v] = nd
                heapq.heappush(heap, (nd, v))
    return np.array([U if x is None else x for x in dist], dtype=np.uint32)


def dijkstra_scipy(g, src):
    w = g.w.astype(np.float64) if g.w is not None else np.ones(g.m)
    srcs = np.repeat(np.arange(g.n), g.outdeg)
    a = csr_matrix((w, (srcs, g.dst)), shape=(g.n, g.n))  # no duplicates after clean-up
    d = dijkstra(a, directed=True, indices=src)
    out = np.full(g.n, U, dtype=np.uint32)
    fin = np.isfinite(d)
    out[fin] = d[fin].astype(np.uint32)
    return out


def transition_matrix(n, off, dst):
    """P[u, v] = multiplicity(u -> v) / outdeg(u); zero rows for dangling u."""
    off = np.asarray(off, dtype=np.int64)
    deg = np.diff(off)
    srcs = np.repeat(np.arange(n), deg)
    p = np.zeros((n, n))
    np.add.at(p, (srcs, np.asarray(dst)), 1.0 / deg[srcs])
    return p


def pagerank_matrix_power(n, off, dst, T, d=D, source=None):
    """r(T) = sum_{k<T} (d P^T)^k t + (d P^T)^T r(0), evaluated with matrix powers."""
    a = d * transition_matrix(n, off, dst).T
    if source is None:
        t = np.full(n, (1 - d) / n)
        r0 = np.full(n, 1.0 / n)
    else:
        t = np.zeros(n)
        t[source] = 1 - d
        r0 = np.zeros(n)
        r0[source] = 1.0
    acc = np.zeros(n)
    for k in range(T):
        acc += np.linalg.matrix_power(a, k) @ t
    return acc + np.linalg.matrix_power(a, T) @ r0


def pagerank_fraction(n, off, dst, T, d=Fraction(17, 20), source=None):
    """Exact rational PageRank iteration (d = 17/20 = 0.85)."""
    off = [int(x) for x in off]
    r = [Fraction(1, n)] * n if source is None else [Fraction(int(v == source)) for v in range(n)]
    for _ in range(T):
        acc = [Fraction(0)] * n
        for u in range(n):
            deg = off[u + 1] - off[u]
            for e in range(off[u], off[u + 1]):
                acc[int(dst[e])] += r[u] / deg
        if source is None:
            r = [(1 - d) / n + d * acc[v] for v in range(n)]
        else:
            r = [(1 - d) * int(v == source) + d * acc[v] for v in range(n)]
    return r


def hop_bounded_min(n, arcs, init, senders0):
    """Synchronous min-plus relaxation in dense form.

    value(s) = min(value(s-1), min_{u->v} value(s-1)[u] + w(u,v)); the vertices
    whose value drops at step s are the step-s senders.  Per step it returns
    the senders, the messages they send (their out-degrees, every arc of a
    multigraph counted: one message per CSR edge, Section V's workload unit)
    and the receivers (vertices with at least one arc from a sender), ending
    as the superstep model ends (see module doc).
    """
    wmat = np.full((n, n), np.inf)
    adj = np.zeros((n, n), dtype=bool)
    outdeg = np.zeros(n, dtype=np.int64)
    for u, v, w in arcs:
        wmat[u, v] = min(wmat[u, v], w)
        adj[u, v] = True
        outdeg[u] += 1
    val = np.array(init, dtype=np.float64)
    sending = senders0.copy()
    senders, messages, receivers = [], [], []

    def record():
        senders.append(int(sending.sum()))
        messages.append(int(outdeg[sending].sum()))
        receivers.append(int(adj[sending].any(axis=0).sum()))

    record()
    while messages[-1] > 0:
        cand = np.min(np.where(sending[:, None], val[:, None] + wmat, np.inf), axis=0)
        new = np.minimum(val, cand)
        sending = new < val
        val = new
        record()
    return senders, messages, receivers


def assert_stats_pinned(r, ref):
    """The oracle's per-superstep senders, messages and receivers against
    hop_bounded_min's (senders, messages, receivers)."""
    senders, messages, receivers = ref
    assert r.senders.tolist() == senders
    assert r.messages.tolist() == messages
    assert r.receivers.tolist() == receivers


def graph_arcs(g, unit=False):
    srcs = np.repeat(np.arange(g.n), g.outdeg)
    ws = np.ones(g.m, dtype=np.int64) if (unit or g.w is None) else g.w.astype(np.int64)
    return list(zip(srcs.tolist(), g.dst.tolist(), ws.tolist()))


# ----------------------------------------------------------------------------- CC

def test_cc_exhaustive_5_vertices():
    pairs = list(itertools.combinations(range(5), 2))
    for mask in range(1 << len(pairs)):
        edges = [pairs[i] for i in range(len(pairs)) if mask >> i & 1]
        g = rmatgen.from_edges(5, [e[0] for e in edges], [e[1] for e in edges], directed=False)
        r = oracle.run_csr("cc", g)
        assert np.array_equal(r.values, union_find_min(5, edges)), edges


@pytest.mark.parametrize("seed", range(6))
def test_cc_random_matches_scipy(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 2048))
    m = int(rng.integers(0, 3 * n))
    s, d = rng.integers(0, n, m), rng.integers(0, n, m)
    g = rmatgen.from_edges(n, s, d, directed=False)
    r = oracle.run_csr("cc", g)
    assert np.array_equal(r.values, min_id_components(n, s, d))
    # label propagation is min-plus relaxation with zero-weight arcs
    zero_arcs = [(u, v, 0) for u, v, _ in graph_arcs(g)]
    assert_stats_pinned(r, hop_bounded_min(n, zero_arcs, np.arange(n), np.ones(n, bool)))


def test_cc_rmat_invariants():
    g = rmatgen.rmat(12, 8, directed=False, seed=3)
    lab = oracle.run_csr("cc", g).values.astype(np.int64)
    v = np.arange(g.n)
    srcs = np.repeat(v, g.outdeg)
    assert np.all(lab <= v)
    assert np.array_equal(lab[lab], lab)
    assert np.array_equal(lab[srcs], lab[g.dst])
    assert np.array_equal(lab, min_id_components(g.n, srcs, g.dst))


@pytest.mark.parametrize("n", [1, 2, 7, 64])
def test_cc_path_closed_form(n):
    r = oracle.run_csr("cc", rmatgen.path(n))
    assert np.all(r.values == 0)
    # vertex k settles at superstep k; one more superstep delivers nothing new
    assert r.supersteps == (n + 1 if n > 1 else 1)
    if n > 1:
        assert r.senders.tolist() == [n - s for s in range(n)] + [0]


def test_cc_cliques_and_isolated():
    g = rmatgen.cliques([3, 1, 4, 2], isolated=3)
    r = oracle.run_csr("cc", g)
    assert r.values.tolist() == [0, 0, 0, 3, 4, 4, 4, 4, 8, 8, 10, 11, 12]
    # a clique settles in one superstep: superstep 1 lowers every non-minimum vertex
    assert r.senders.tolist() == [13, 2 + 3 + 1, 0]


# ----------------------------------------------------------------------------- SSSP

def test_sssp_exhaustive_4_vertex_digraphs():
    arcs_all = [(u, v) for u in range(4) for v in range(4) if u != v]
    rng = np.random.default_rng(11)
    for mask in range(1 << len(arcs_all)):
        arcs = [arcs_all[i] for i in range(len(arcs_all)) if mask >> i & 1]
        g = rmatgen.from_edges(4, [a[0] for a in arcs], [a[1] for a in arcs], directed=True)
        w = rng.integers(1, 256, g.m).astype(np.uint32)
        src = int(rng.integers(0, 4))
        r = oracle.run("sssp", g.n, g.off, g.dst, w, source=src)
        wa = list(zip(np.repeat(np.arange(4), g.outdeg).tolist(), g.dst.tolist(), w.tolist()))
        assert np.array_equal(r.values, dijkstra_heap(4, wa, src)), (arcs, w, src)
        init = np.full(4, np.inf)
        init[src] = 0
        start = np.zeros(4, bool)
        start[src] = True
        ref = hop_bounded_min(4, wa, init, start)
        assert (r.senders.tolist(), r.messages.tolist(), r.receivers.tolist()) == ref, (arcs, w, src)


@pytest.mark.parametrize("seed", range(4))
def test_sssp_rmat_matches_dijkstra(seed):
    g = rmatgen.rmat(11, 8, seed=100 + seed, weighted=True)
    for src in (0, 5, g.n - 1):
        r = oracle.run_csr("sssp", g, source=src)
        ref = dijkstra_scipy(g, src)
        assert np.array_equal(r.values, ref)
        assert r.values[src] == 0
        init = np.full(g.n, np.inf)
        init[src] = 0
        start = np.zeros(g.n, bool)
        start[src] = True
        if seed == 0 and src == 0:
            assert_stats_pinned(r, hop_bounded_min(g.n, graph_arcs(g), init, start))


def test_sssp_unit_weights_are_bfs_levels():
    g = rmatgen.rmat(12, 8, seed=5)
    srcs = np.repeat(np.arange(g.n), g.outdeg)
    a = csr_matrix((np.ones(g.m), (srcs, g.dst)), shape=(g.n, g.n))
    lev = shortest_path(a, directed=True, unweighted=True, indices=0)
    r = oracle.run_csr("sssp", g, source=0)  # no weight array: unit weights
    fin = np.isfinite(lev)
    assert np.array_equal(r.values[fin], lev[fin].astype(np.uint32))
    assert np.all(r.values[~fin] == U)
    # frontier of superstep s = BFS level s
    order = breadth_first_order(a, 0, directed=True, return_predecessors=False)
    sizes = np.bincount(lev[order].astype(np.int64))
    assert r.senders[: len(sizes)].tolist() == sizes.tolist()


def test_sssp_weighted_path_prefix_sums_and_unreachable():
    n = 9
    w = np.array([3, 1, 255, 7, 2, 9, 4, 1], dtype=np.uint32)
    g = rmatgen.raw_csr(n + 2, np.arange(n - 1), np.arange(1, n), w)  # two isolated vertices at the end
    r = oracle.run("sssp", g.n, g.off, g.dst, g.w, source=0)
    assert r.values[:n].tolist() == [0] + np.cumsum(w).tolist()
    assert r.values[n:].tolist() == [U, U]
    r = oracle.run("sssp", g.n, g.off, g.dst, g.w, source=4)
    assert r.values[:4].tolist() == [U] * 4
    assert r.values[4:n].tolist() == [0] + np.cumsum(w[4:]).tolist()


def test_sssp_multigraph_takes_lightest_parallel_edge():
    g = rmatgen.raw_csr(3, [0, 0, 0, 1, 1], [1, 1, 2, 2, 1], [9, 4, 20, 3, 1])
    r = oracle.run("sssp", g.n, g.off, g.dst, g.w, source=0)
    assert r.values.tolist() == [0, 4, 7]


# ----------------------------------------------------------------------------- PageRank / PPR

def test_pagerank_exact_rationals_all_4_vertex_digraphs():
    arcs_all = [(u, v) for u in range(4) for v in range(4) if u != v]
    for mask in range(0, 1 << len(arcs_all), 7):  # 586 of the 4,096 digraphs
        arcs = [arcs_all[i] for i in range(len(arcs_all)) if mask >> i & 1]
        g = rmatgen.from_edges(4, [a[0] for a in arcs], [a[1] for a in arcs], directed=True)
        for T in (1, 3):
            got = oracle.run_csr("pagerank", g, T=T).values
            exact = pagerank_fraction(4, g.off, g.dst, T)
            assert np.allclose(got, [float(x) for x in exact], rtol=0, atol=1e-15), (arcs, T)


def test_pagerank_exact_rationals_multigraph_with_self_loops():
    # every CSR entry is an edge: multiplicities count in the out-degree and the sums
    g = rmatgen.raw_csr(4, [0, 0, 0, 1, 1, 2, 3, 3], [1, 1, 0, 2, 2, 2, 0, 1])
    got = oracle.run("pagerank", g.n, g.off, g.dst, T=4).values
    exact = pagerank_fraction(4, g.off, g.dst, 4)
    assert np.allclose(got, [float(x) for x in exact], rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", range(5))
@pytest.mark.parametrize("T", [0, 1, 2, 10, 20])
def test_pagerank_matches_matrix_power(seed, T):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 400))
    m = int(rng.integers(0, 6 * n))
    g = rmatgen.raw_csr(n, rng.integers(0, n, m), rng.integers(0, n, m))
    got = oracle.run("pagerank", n, g.off, g.dst, T=T)
    assert np.max(np.abs(got.values - pagerank_matrix_power(n, g.off, g.dst, T))) <= 1e-12
    src = int(rng.integers(0, n))
    got = oracle.run("ppr", n, g.off, g.dst, T=T, source=src)
    assert np.max(np.abs(got.values - pagerank_matrix_power(n, g.off, g.dst, T, source=src))) <= 1e-12


@pytest.mark.parametrize("n", [2, 5, 1000])
def test_pagerank_cycle_and_complete_are_uniform(n):
    for T in (1, 10):
        assert np.allclose(oracle.run_csr("pagerank", rmatgen.cycle(n), T=T).values, 1.0 / n, rtol=1e-14)
    if n <= 50:
        assert np.allclose(oracle.run_csr("pagerank", rmatgen.complete_digraph(n), T=7).values, 1.0 / n, rtol=1e-14)


@pytest.mark.parametrize("L", [1, 3, 100])
def test_pagerank_star_closed_forms(L):
    n = L + 1
    base = (1 - D) / n
    for T in (1, 2, 5):
        out = oracle.run_csr("pagerank", rmatgen.out_star(L), T=T).values
        assert out[0] == pytest.approx(base, rel=1e-14)
        leaf = base + D / (n * L) if T == 1 else base + D * base / L
        assert np.allclose(out[1:], leaf, rtol=1e-14)
        inn = oracle.run_csr("pagerank", rmatgen.in_star(L), T=T).values
        assert np.allclose(inn[1:], base, rtol=1e-14)
        hub = base + D * L / n if T == 1 else base + D * L * base
        assert inn[0] == pytest.approx(hub, rel=1e-14)
    # bidirectional star: 2x2 recurrence, total mass stays 1
    h, l = 1.0 / n, 1.0 / n
    for T in range(1, 8):
        h, l = base + D * L * l, base + D * h / L
        bi = oracle.run_csr("pagerank", rmatgen.bi_star(L), T=T).values
        assert bi[0] == pytest.approx(h, rel=1e-13)
        assert np.allclose(bi[1:], l, rtol=1e-13)
        assert bi.sum() == pytest.approx(1.0, rel=1e-13)


def test_pagerank_dangling_mass_invariant_and_stats():
    g = rmatgen.rmat(12, 8, seed=9)
    deg = g.outdeg
    prev = None
    for T in range(0, 6):
        r = oracle.run_csr("pagerank", g, T=T)
        if prev is not None:
            assert r.values.sum() == pytest.approx((1 - D) + D * prev[deg > 0].sum(), rel=1e-12)
        prev = r.values
        assert r.supersteps == T + 1
        assert r.senders.tolist() == [g.n] * T + [0]
        assert r.messages.tolist() == [g.m] * T + [0]
        indeg_pos = int((np.bincount(g.dst, minlength=g.n) > 0).sum())
        assert r.receivers.tolist() == [indeg_pos] * T + [0]


# ----------------------------------------------------------------------------- argument checking

def test_oracle_rejects_bad_source():
    g = rmatgen.path(3)
    with pytest.raises(oracle.OracleError):
        oracle.run_csr("sssp", g, source=3)
    with pytest.raises(oracle.OracleError):
        oracle.run_csr("ppr", g, source=-1)


def test_oracle_reports_cap():
    g = rmatgen.path(10)
    with pytest.raises(oracle.OracleError):
        oracle.run_csr("cc", g, max_supersteps=5)


# ---------------------------------------------------------------- combiners
# One superstep of message passing with a chosen combiner (paper, Section III
# and Figure 1: the first message is stored, later ones merged; no neutral
# value).  Pinned against numpy's unbuffered ufunc.at, which applies an
# operation at repeated indices one at a time in index order, and against
# brute force over each receiver's sorted incoming messages.

def _edges(g):
    src = np.repeat(np.arange(g.n), np.diff(g.off))
    return src, np.asarray(g.dst, dtype=np.int64)


def _combine_case(seed):
    g = rmatgen.rmat(9, 6, seed=seed)
    rng = np.random.default_rng(seed)
    active = rng.random(g.n) < 0.7
    return g, rng, active


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_combine_integer_sum_and_product_match_ufunc_at(seed):
    g, rng, active = _combine_case(seed)
    msg = rng.integers(0, 2**64, g.n, dtype=np.uint64)
    src, dst = _edges(g)
    keep = active[src]
    counts = np.bincount(dst[keep], minlength=g.n)
    box, has = oracle.combine("sum_u64", g.n, g.off, g.dst, msg, active)
    ref = np.zeros(g.n, np.uint64)
    np.add.at(ref, dst[keep], msg[src[keep]])
    assert np.array_equal(has, counts > 0) and np.array_equal(box[has], ref[has])
    # product: a neutral-initialised mailbox would agree (1 * x = x); a
    # zero-initialised one would not, and the flags must still match
    box, has = oracle.combine("prod_u64", g.n, g.off, g.dst, msg | np.uint64(1), active)
    ref = np.ones(g.n, np.uint64)
    np.multiply.at(ref, dst[keep], (msg | np.uint64(1))[src[keep]])
    assert np.array_equal(has, counts > 0) and np.array_equal(box[has], ref[has])


@pytest.mark.parametrize("seed", [4, 5])
def test_combine_float_max_and_ordered_sum(seed):
    g, rng, active = _combine_case(seed)
    vals = rng.standard_normal(g.n)
    src, dst = _edges(g)
    keep = active[src]
    box, has = oracle.combine("max_f64", g.n, g.off, g.dst, vals, active)
    ref = np.full(g.n, -np.inf)
    np.maximum.at(ref, dst[keep], vals[src[keep]])
    assert np.array_equal(box.view(np.float64)[has], ref[has])
    # sum in sender order: identical bits to sequential ufunc.at from +0.0
    # (no message is -0.0, so the stored first message equals 0.0 + it)
    box, has = oracle.combine("sum_f64", g.n, g.off, g.dst, vals, active)
    ref = np.zeros(g.n)
    np.add.at(ref, dst[keep], vals[src[keep]])
    assert np.array_equal(box.view(np.float64)[has], ref[has])
    assert not has[np.bincount(dst[keep], minlength=g.n) == 0].any()


def load_golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)) as f:
        return json.load(f)


def test_combine_golden_neutral_combination():
    """Section III's case, written out by hand (tests/golden): messages whose
    combination equals the combiner's neutral value still leave the receiver
    with a message, and a receiver whose only sender is inactive has none."""
    fx = load_golden("neutral_combination.json")
    gr = fx["graph"]
    active = np.array(gr["active"], bool)
    for case in fx["cases"]:
        msg = np.array([int(x, 16) for x in case["msg"]], np.uint64)
        box, has = oracle.combine(case["op"], gr["n"], gr["off"], gr["dst"], msg, active)
        assert has.tolist() == [bool(h) for h in case["has"]], case["op"]
        for v, want in enumerate(case["box"]):
            if want is not None:
                assert int(box[v]) == int(want, 16), (case["op"], v)


def _pack(val32, ids):
    return (ids.astype(np.uint64) << np.uint64(32)) | val32.view(np.uint32).astype(np.uint64)


@pytest.mark.parametrize("seed", [6, 7])
def test_combine_minarg_brute_force_with_ties(seed):
    g, rng, active = _combine_case(seed)
    vals = rng.integers(-3, 4, g.n).astype(np.float32)  # many ties
    ids = rng.permutation(g.n).astype(np.uint32)
    box, has = oracle.combine("minarg", g.n, g.off, g.dst, _pack(vals, ids), active)
    src, dst = _edges(g)
    for u in range(g.n):
        senders = src[(dst == u) & active[src]]
        assert has[u] == (senders.size > 0)
        if senders.size:
            best = min(senders, key=lambda v: (vals[v], ids[v]))
            assert box[u] == _pack(vals[best:best + 1], ids[best:best + 1])[0], u


def test_combine_inactive_and_duplicate_edges():
    c = rmatgen.raw_csr(4, [0, 0, 1, 3, 3], [1, 1, 1, 1, 2])
    msg = np.array([3, 5, 7, 11], np.uint64)
    box, has = oracle.combine("prod_u64", 4, c.off, c.dst, msg, np.array([1, 1, 0, 1]))
    assert has.tolist() == [False, True, True, False]
    assert box[1] == 3 * 3 * 5 * 11 and box[2] == 11
    box, has = oracle.combine("sum_u64", 4, c.off, c.dst, msg)
    assert box[1] == 3 + 3 + 5 + 11 and box[2] == 11
    with pytest.raises(oracle.OracleError):
        oracle.combine(9, 4, c.off, c.dst, msg)
