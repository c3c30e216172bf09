"""HIP path vs the CPU oracle on small and mid-size graphs (GPU).

Sizes span several merge-path tiles with ragged tails; every program runs
under both work distributions, int32 and int64 offsets, unit and uint32
weights; edge cases include empty graphs, isolated vertices, sources without
out-edges, hubs longer than a tile, multigraphs and self-loops.
"""
import numpy as np
import pytest

import rmatgen
from gpu_util import check_min, check_rank, run_gpu

pytestmark = pytest.mark.gpu

SCHEDS = ["vertex", "edge", "pull", "auto"]


def make(csr, **kw):
    from paper_2010_01542_amd import Graph
    return Graph.from_csr(csr, **kw)


def hand_graphs():
    return {
        "single": rmatgen.raw_csr(1, [], []),
        "isolated100": rmatgen.raw_csr(100, [], []),
        "path2": rmatgen.path(2),
        "path60": rmatgen.path(60),
        "cycle7": rmatgen.cycle(7),
        "outstar5000": rmatgen.out_star(5000),
        "instar5000": rmatgen.in_star(5000),
        "bistar300": rmatgen.bi_star(300),
        "cliques": rmatgen.cliques([3, 1, 40, 2], isolated=5),
        "complete40": rmatgen.complete_digraph(40),
        "multigraph": rmatgen.raw_csr(6, [0, 0, 0, 1, 1, 2, 3, 3, 5, 5], [1, 1, 0, 2, 2, 2, 0, 1, 5, 4],
                                      [5, 2, 1, 9, 3, 7, 1, 1, 4, 250]),
    }


@pytest.fixture(scope="module")
def hand(device):
    gs = hand_graphs()
    return {(k, rl): (c, make(c, relabel=rl)) for k, c in gs.items() for rl in (True, False)}


@pytest.mark.parametrize("relabel", [True, False])
@pytest.mark.parametrize("sched", SCHEDS)
@pytest.mark.parametrize("name", sorted(hand_graphs()))
def test_hand_graphs_all_programs(hand, name, sched, relabel):
    csr, g = hand[(name, relabel)]
    print(f"case hand/{name}/{sched}/relabel={relabel}", flush=True)
    sym = rmatgen.from_edges(csr.n, np.repeat(np.arange(csr.n), csr.outdeg), csr.dst, directed=False)
    check_min(sym, make(sym, relabel=relabel), "cc", schedule=sched)
    check_min(sym, make(sym, symmetric=True, relabel=relabel), "cc", schedule=sched)
    for src in sorted({0, csr.n - 1}):
        check_min(csr, g, "sssp", source=src, schedule=sched)
    check_rank(csr, g, "pagerank", T=10, schedule=sched)
    check_rank(csr, g, "ppr", T=7, source=0, schedule=sched)


@pytest.mark.parametrize("tile", [64, 256, 2048, 8192])
@pytest.mark.parametrize("off_dtype", [np.int32, np.int64])
@pytest.mark.parametrize("seed", [1, 2])
def test_rmat_tiles_offsets(device, tile, off_dtype, seed):
    print(f"case rmat s12 tile={tile} off={np.dtype(off_dtype).name} seed={seed}", flush=True)
    d = rmatgen.rmat(12, 16, seed=seed, weighted=True, offset_dtype=off_dtype)
    u = rmatgen.rmat(12, 16, seed=seed, directed=False, offset_dtype=off_dtype)
    gd, gu = make(d, relabel=seed == 1), make(u, relabel=seed == 1)
    for sched in ("vertex", "edge", "pull"):
        check_min(d, gd, "sssp", source=0, schedule=sched, tile=tile)
        check_min(u, gu, "cc", schedule=sched, tile=tile)
        check_rank(d, gd, "pagerank", T=10, schedule=sched, tile=tile)
    check_min(u, make(u, symmetric=True), "cc", schedule="pull", tile=tile)


@pytest.mark.parametrize("scale,ef", [(10, 4), (14, 8), (16, 16), (18, 16)])
def test_rmat_sizes(device, scale, ef):
    print(f"case rmat scale={scale} ef={ef}", flush=True)
    d = rmatgen.rmat(scale, ef, seed=scale, weighted=True)
    gd = make(d)
    for src in (0, 3, d.n - 1):
        check_min(d, gd, "sssp", source=src)
    u = rmatgen.rmat(scale, ef, seed=scale + 50, directed=False, offset_dtype=np.int32)
    check_min(u, make(u), "cc")
    unit = rmatgen.Csr(d.n, d.m, d.off, d.dst, None)
    check_min(unit, make(unit), "sssp", source=0)  # unit weights = BFS levels
    check_rank(d, gd, "pagerank", T=20)
    check_rank(d, gd, "ppr", T=20, source=1)


def test_schedules_agree_exactly_on_min_programs(device):
    u = rmatgen.rmat(15, 16, seed=77, directed=False)
    g = make(u)
    a, sa = run_gpu(g, "cc", schedule="vertex")
    b, sb = run_gpu(g, "cc", schedule="edge", tile=512)
    c, sc = run_gpu(g, "cc", schedule="pull", tile=1024)
    assert np.array_equal(a, b) and sa.frontier.tolist() == sb.frontier.tolist()
    assert np.array_equal(a, c) and sa.frontier.tolist() == sc.frontier.tolist()


def test_test_before_atomic_is_a_pure_optimisation(device):
    from paper_2010_01542_amd import vc
    d = rmatgen.rmat(14, 16, seed=3, weighted=True)
    g = make(d)
    a, sa = run_gpu(g, "sssp", source=0)
    b, sb = run_gpu(g, "sssp", source=0, options=vc.OPT_NO_TEST_BEFORE_ATOMIC)
    assert np.array_equal(a, b) and sa.frontier.tolist() == sb.frontier.tolist()


def test_repeated_runs_reuse_workspace(device):
    d = rmatgen.rmat(13, 8, seed=5, weighted=True)
    g = make(d)
    first = run_gpu(g, "sssp", source=0)[0]
    run_gpu(g, "pagerank", T=3)
    run_gpu(g, "cc")
    again = run_gpu(g, "sssp", source=0)[0]
    assert np.array_equal(first, again)


def test_copy_mode_and_validation(device):
    import torch
    from paper_2010_01542_amd import Graph, VcError
    d = rmatgen.rmat(11, 8, seed=8, weighted=True)
    off = torch.from_numpy(d.off).cuda()
    dst = torch.from_numpy(d.dst).cuda()
    w = torch.from_numpy(d.w.view(np.int32)).cuda()
    g = Graph(off, dst, w, borrow=False, validate=True)
    del off, dst, w
    torch.cuda.synchronize()
    check_min(d, g, "sssp", source=0)
    bad = d.dst.copy()
    bad[17] = d.n  # out of range
    with pytest.raises(VcError):
        Graph(torch.from_numpy(d.off).cuda(), torch.from_numpy(bad).cuda(), None, validate=True)
    off_bad = d.off.copy()
    off_bad[-1] -= 1
    with pytest.raises(VcError):
        Graph(torch.from_numpy(off_bad).cuda(), torch.from_numpy(d.dst).cuda(), None, validate=True)


def test_argument_errors(device):
    from paper_2010_01542_amd import VcError
    g = make(rmatgen.path(4, directed=True))
    with pytest.raises(VcError):
        g.run("sssp", source=4)
    with pytest.raises(VcError):
        g.run("pagerank", T=-1)
    with pytest.raises(VcError):
        g.run("pagerank", damping=1.5)


def test_superstep_cap(device):
    from paper_2010_01542_amd import VcError, vc
    g = make(rmatgen.path(50))
    with pytest.raises(VcError) as e:
        g.run("cc", max_supersteps=10)
    assert e.value.status == vc.ERR_NOT_CONVERGED


def test_timing_stats_are_recorded(device):
    d = rmatgen.rmat(14, 16, seed=2, weighted=True)
    g = make(d)
    _, st = g.run("pagerank", T=5, timing=True, schedule="pull")  # eager loop: every kernel timed
    assert st.scatter_ms.shape[0] == 6 and np.all(st.scatter_ms[:5] > 0) and np.all(st.step_ms[:5] >= st.scatter_ms[:5])
    # AUTO on a small graph captures the loop: the graph's time averaged over the supersteps
    _, st = g.run("pagerank", T=5, timing=True)
    assert np.all(st.scatter_ms[:5] == 0) and np.all(st.step_ms[:5] > 0) and np.ptp(st.step_ms[:5]) == 0
    _, st = g.run("sssp", source=0, timing=True)
    assert np.all(st.scatter_ms[: st.supersteps - 1] > 0)


def test_fixed_point_pagerank_is_order_independent(device):
    d = rmatgen.rmat(15, 16, seed=4)
    g = make(d)
    a = run_gpu(g, "pagerank", T=10, schedule="vertex")[0]
    b = run_gpu(g, "pagerank", T=10, schedule="edge", tile=256)[0]
    c = run_gpu(g, "pagerank", T=10, schedule="edge", tile=4096)[0]
    d2 = run_gpu(g, "pagerank", T=10, schedule="pull", tile=512)[0]
    e = run_gpu(g, "pagerank", T=10, schedule="blocked")[0]
    assert np.array_equal(a, b) and np.array_equal(a, c) and np.array_equal(a, d2) and np.array_equal(a, e)


@pytest.mark.parametrize("relabel", [True, False])
def test_blocked_pagerank_matches_oracle_and_pull(device, relabel):
    """Propagation blocking: several source tiles (2^18 vertices each), bins
    split over several fold items (hot destinations), vertices without
    out-edges, PPR from a hub; ranks equal the pull form's bit for bit."""
    print(f"case blocked pagerank s19 relabel={relabel}", flush=True)
    d = rmatgen.rmat(19, 12, seed=8)
    g = make(d, relabel=relabel)
    check_rank(d, g, "pagerank", T=4, schedule="blocked")
    check_rank(d, g, "ppr", T=5, source=0, schedule="blocked")
    a = run_gpu(g, "pagerank", T=6, schedule="blocked")[0]
    b = run_gpu(g, "pagerank", T=6, schedule="pull")[0]
    assert np.array_equal(a, b)
    for c in (rmatgen.in_star(40000), rmatgen.cycle(5), rmatgen.raw_csr(6, [0, 0, 1, 5, 5], [1, 1, 1, 0, 2]),
              rmatgen.raw_csr(7, [], [])):
        check_rank(c, make(c, relabel=relabel), "pagerank", T=3, schedule="blocked")


@pytest.mark.parametrize("relabel", [True, False])
def test_blocked_pagerank_every_kind_of_bin(device, relabel):
    """Destination bins of the blocked form come in three kinds: one fold
    item (mailboxes stored), split over several items (mailboxes added) and
    without in-edges (no item).  R-MAT plus a tail of isolated vertices
    (three empty bins and a ragged last one) has all three in either vertex
    order (int32 offsets when not relabelled).  Ranks equal the pull form's
    bit for bit at every T from 1 to 3 for both message kinds, for PPR from
    a hub, from a vertex without in-edges and from an isolated one, and for
    runs that follow each other on one graph (a last superstep leaves its
    sums in the mailboxes)."""
    from paper_2010_01542_amd import vc
    print(f"case blocked pagerank every kind of bin relabel={relabel}", flush=True)
    r = rmatgen.rmat(17, 8, seed=3)
    src = np.repeat(np.arange(r.n), np.diff(np.asarray(r.off, np.int64)))
    d = rmatgen.raw_csr(r.n + 3 * 4096 + 100, src, r.dst, offset_dtype=np.int64 if relabel else np.int32)
    g = make(d, relabel=relabel)
    for T in (1, 2, 3):
        for opt in (0, vc.OPT_F32_MESSAGES):
            a = run_gpu(g, "pagerank", T=T, schedule="blocked", options=opt)[0]
            b = run_gpu(g, "pagerank", T=T, schedule="pull", options=opt)[0]
            assert np.array_equal(a, b), (T, opt)
    indeg = np.bincount(np.asarray(d.dst), minlength=d.n)
    for s in (int(indeg.argmax()), int(np.flatnonzero(indeg == 0)[0]), d.n - 1):
        a = run_gpu(g, "ppr", T=4, source=s, schedule="blocked")[0]
        b = run_gpu(g, "ppr", T=4, source=s, schedule="pull")[0]
        assert np.array_equal(a, b), s
    check_rank(d, g, "pagerank", T=5, schedule="blocked")


@pytest.mark.parametrize("relabel", [True, False])
def test_f32_messages_meet_tolerance_and_agree_across_schedules(device, relabel):
    """Binary32 messages summed exactly in fixed point: within the PageRank
    bars of the oracle, and one result for every schedule (each message is
    rounded once, then the sum is exact in any order), captured or not."""
    from paper_2010_01542_amd import vc
    print(f"case f32 messages s19 relabel={relabel}", flush=True)
    d = rmatgen.rmat(19, 12, seed=8)
    g = make(d, relabel=relabel)
    opt = vc.OPT_F32_MESSAGES
    outs = [check_rank(d, g, "pagerank", T=6, schedule=s, options=opt)[0]
            for s in ("vertex", "edge", "pull", "blocked", "auto")]
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)
    cap = run_gpu(g, "pagerank", T=6, schedule="blocked", options=opt | vc.OPT_GRAPH_CAPTURE)[0]
    assert np.array_equal(outs[0], cap)
    ppr = [check_rank(d, g, "ppr", T=6, source=0, schedule=s, options=opt)[0] for s in ("pull", "blocked")]
    assert np.array_equal(ppr[0], ppr[1])
    # the one extra rounding per message moves ranks by far less than the bars
    fixed = run_gpu(g, "pagerank", T=6)[0].astype(np.float64)
    assert np.abs(outs[0] - fixed).max() <= 4 * np.spacing(np.float32(fixed.max()))


def test_f32_options_exclude_each_other(device):
    from paper_2010_01542_amd import VcError, vc
    g = make(rmatgen.cycle(8))
    with pytest.raises(VcError):
        g.run("pagerank", options=vc.OPT_F32_MESSAGES | vc.OPT_F32_ACCUMULATE)


def test_blocked_schedule_rejects_f32_atomics(device):
    from paper_2010_01542_amd import VcError, vc
    g = make(rmatgen.path(8, directed=True))
    with pytest.raises(VcError):
        g.run("pagerank", schedule="blocked", options=vc.OPT_F32_ACCUMULATE)


@pytest.mark.parametrize("relabel", [True, False])
def test_blocked_min_programs_bit_exact(device, relabel):
    """Every superstep of CC / SSSP in the blocked form (spread of each slot's
    message, LDS minima per destination bin, the pull form's mailbox and
    improvement rule): values, superstep counts and per-superstep frontier
    and message counts equal the oracle's.  Several source tiles, bins split
    over items (hubs), weighted, unit-weight and symmetric graphs."""
    print(f"case blocked min programs s19 relabel={relabel}", flush=True)
    dw = rmatgen.rmat(19, 8, seed=12, weighted=True)
    gw = make(dw, relabel=relabel)
    for src in (0, 77):
        check_min(dw, gw, "sssp", source=src, schedule="blocked")
    du = rmatgen.rmat(18, 8, seed=13)
    check_min(du, make(du, relabel=relabel), "sssp", source=3, schedule="blocked")
    sym = rmatgen.rmat(18, 8, seed=14, directed=False)
    check_min(sym, make(sym, symmetric=True, relabel=relabel), "cc", schedule="blocked")
    for c in (rmatgen.in_star(40000), rmatgen.path(9, directed=True), rmatgen.cycle(5),
              rmatgen.raw_csr(6, [0, 0, 1, 5, 5], [1, 1, 1, 0, 2]), rmatgen.raw_csr(7, [], [])):
        check_min(c, make(c, relabel=relabel), "sssp", source=0, schedule="blocked")
        check_min(c, make(c, relabel=relabel), "cc", schedule="blocked")
    # weights beyond one byte: the layout keeps them 4 bytes wide
    big = rmatgen.Csr(dw.n, dw.m, dw.off, dw.dst, (dw.w.astype(np.uint32) * np.uint32(1000)).astype(np.uint32))
    check_min(big, make(big, relabel=relabel), "sssp", source=0, schedule="blocked")


def test_blocked_sssp_slot_width_switch(device):
    """Single-source SSSP's blocked supersteps carry messages in 2-byte slots
    while every message of the superstep is bounded below 0xFFFF ((superstep
    + 1) times the largest weight) and in 4-byte slots after: a weighted path
    whose distances pass 65,535 switches width in mid-run; an R-MAT graph
    with weights up to 30,000 switches after two supersteps; one with
    weights beyond 65,535 never narrows.  Bit-exact against the oracle."""
    print("case blocked SSSP slot width switch", flush=True)
    n = 300
    path = rmatgen.raw_csr(n, np.arange(n - 1), np.arange(1, n), np.full(n - 1, 997, np.uint32))
    check_min(path, make(path), "sssp", source=0, schedule="blocked")
    check_min(path, make(path, relabel=False), "sssp", source=5, schedule="blocked")
    d = rmatgen.rmat(16, 8, seed=41, weighted=True)
    rng = np.random.default_rng(41)
    for top in (30000, 1 << 20):
        c = rmatgen.Csr(d.n, d.m, d.off, d.dst, rng.integers(1, top, d.m, dtype=np.uint32))
        check_min(c, make(c), "sssp", source=0, schedule="blocked")
        check_min(c, make(c), "sssp", source=0)  # AUTO: push and pull at this size


def test_auto_takes_the_blocked_form_for_dense_min_supersteps(device):
    print("case auto blocked min s20", flush=True)
    d = rmatgen.rmat(20, 8, seed=15, weighted=True)
    g = make(d)
    got, st, ref = check_min(d, g, "sssp", source=0)
    assert 4 in set(st.schedule.tolist()), st.schedule
    sym = rmatgen.rmat(20, 4, seed=16, directed=False)
    got, st, ref = check_min(sym, make(sym, symmetric=True), "cc")
    assert 4 in set(st.schedule.tolist()), st.schedule


@pytest.mark.parametrize("program", ["pagerank", "ppr"])
def test_fixed_point_rank_within_one_ulp_of_oracle(device, program):
    import oracle
    d = rmatgen.rmat(14, 16, seed=6)
    ref = oracle.run_csr(program, d, T=10, source=2).values
    got = run_gpu(make(d), program, T=10, source=2)[0]
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(got.astype(np.float64) - ref) <= ulp)


@pytest.mark.parametrize("scale", [12, 16])
def test_f32_accumulate_meets_tolerance_on_rmat(device, scale):
    from paper_2010_01542_amd import vc
    d = rmatgen.rmat(scale, 16, seed=scale)
    g = make(d)
    for sched in ("vertex", "edge", "pull"):
        check_rank(d, g, "pagerank", T=10, schedule=sched, options=vc.OPT_F32_ACCUMULATE)


def test_auto_schedule_mixes_push_and_pull(device):
    d = rmatgen.rmat(16, 16, seed=21, weighted=True)
    got, st, ref = check_min(d, make(d), "sssp", source=0, schedule="auto")
    used = set(st.schedule.tolist())
    assert 3 in used and (1 in used or 2 in used), used


def test_relabelled_and_input_order_agree_bit_for_bit(device):
    d = rmatgen.rmat(15, 16, seed=31, weighted=True)
    a, b = make(d, relabel=True), make(d, relabel=False)
    for prog, kw in (("sssp", dict(source=7)), ("cc", {}), ("pagerank", dict(T=10)), ("ppr", dict(T=10, source=7))):
        x, sx = run_gpu(a, prog, **kw)
        y, sy = run_gpu(b, prog, **kw)
        assert np.array_equal(x, y), prog
        assert sx.frontier.tolist() == sy.frontier.tolist(), prog
