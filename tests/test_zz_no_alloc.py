"""vc_run_noalloc (the entry point that allocates nothing) against vc_run.

Through the C ABI, on the GPU: every program's result from the fixed
workspace equals vc_run's on the same graph and params (bit for bit: CC
labels, SSSP distances, fixed-point PageRank / PPR ranks), with the same
per-superstep frontier sizes and message counts; two calls in a row, the
second on a smaller graph, so that the second run finds the first one's data
in the shared workspace; a graph never prepared (AUTO then pushes); and the
refusals: a graph whose workspace exceeds the fixed size, the blocked form,
captured loops, and an explicit pull without the transpose.
"""
import numpy as np
import pytest

import rmatgen

pytestmark = pytest.mark.gpu


def make(csr, **kw):
    from paper_2010_01542_amd import Graph
    return Graph.from_csr(csr, **kw)


def host(out):
    v = out.cpu().numpy()
    return v.view(np.uint32) if v.dtype == np.int32 else v


def both(g, program, **kw):
    """(vc_run result, stats), (vc_run_noalloc result, stats)."""
    import torch
    rank = program in ("pagerank", "ppr")
    dt = torch.float32 if rank else torch.int32
    a, sa = g.run(program, torch.empty(g.n, dtype=dt, device="cuda"), stats=True, **kw)
    out = torch.full((g.n,), 7, dtype=dt, device="cuda")  # stale contents must not matter
    b, sb = g.run_noalloc(program, out, stats=True, **kw)
    return (host(a), sa), (host(b), sb)


def same(program, g, **kw):
    (a, sa), (b, sb) = both(g, program, **kw)
    assert np.array_equal(a, b), (program, kw, int((a != b).sum()))
    assert sb.supersteps == sa.supersteps
    if program in ("cc", "sssp"):
        assert sb.frontier.tolist() == sa.frontier.tolist()
        assert sb.edges.tolist() == sa.edges.tolist()
    return b


PROGRAMS = [("sssp", dict(source=5)), ("cc", {}), ("pagerank", dict(T=10)), ("ppr", dict(T=12, source=3)),
            ("pagerank", dict(T=6, options=16))]  # options=16: binary32 messages


def test_two_calls_in_a_row_second_smaller(device):
    from paper_2010_01542_amd import vc
    big_d = rmatgen.rmat(15, 16, seed=41, weighted=True)
    big_u = rmatgen.rmat(15, 16, seed=42, directed=False)
    small_d = rmatgen.rmat(9, 4, seed=43, weighted=True)
    small_u = rmatgen.rmat(9, 4, seed=44, directed=False)
    graphs = {"big": (make(big_d), make(big_u, symmetric=True)), "small": (make(small_d), make(small_u, symmetric=True))}
    for gd, gu in graphs.values():
        for prog, kw in PROGRAMS:
            (gu if prog == "cc" else gd).prepare(prog, **{k: v for k, v in kw.items() if k in ("T", "source", "options")})
    for size in ("big", "small", "big"):
        gd, gu = graphs[size]
        for prog, kw in PROGRAMS:
            print(f"case noalloc {size} {prog} {kw}", flush=True)
            same(prog, gu if prog == "cc" else gd, **kw)
    # explicit push schedules too, with and without hub aggregation
    gd, gu = graphs["small"]
    for sched in ("vertex", "edge", "pull"):
        for opt in (0, vc.OPT_NO_HUB_AGGREGATION):
            print(f"case noalloc small schedule={sched} options={opt}", flush=True)
            same("sssp", gd, source=0, schedule=sched, options=opt)
            same("cc", gu, schedule=sched, options=opt)


def test_unprepared_graph_pushes(device):
    """Nothing built yet: AUTO takes the push forms (vertex-per-thread for
    dense supersteps, since the CSR partition is missing either)."""
    from paper_2010_01542_amd import vc
    d = rmatgen.rmat(12, 8, seed=45, weighted=True)
    g = make(d)
    import torch
    out = torch.empty(d.n, dtype=torch.int32, device="cuda")
    b, sb = g.run_noalloc("sssp", out, source=0, stats=True)
    assert vc.SCHED_PULL not in sb.schedule.tolist() and vc.SCHED_BLOCKED not in sb.schedule.tolist()
    a, sa = g.run("sssp", source=0, stats=True)
    assert np.array_equal(host(a), host(b))
    assert sa.edges.tolist() == sb.edges.tolist()
    u = rmatgen.rmat(12, 8, seed=46, directed=False)
    gu = make(u, symmetric=True)
    b, sb = gu.run_noalloc("cc", torch.empty(u.n, dtype=torch.int32, device="cuda"), stats=True)
    assert sb.schedule.tolist()[0] == vc.SCHED_VERTEX
    assert np.array_equal(host(gu.run("cc")[0]), host(b))
    r = torch.empty(d.n, dtype=torch.float32, device="cuda")
    assert np.array_equal(host(g.run("pagerank", T=5)[0]), host(g.run_noalloc("pagerank", r, T=5)[0]))


def test_refusals(device):
    import torch
    from paper_2010_01542_amd import VcError, vc
    print("case noalloc refusals", flush=True)
    n = 5_000_000  # CC / SSSP need ~20 bytes and PageRank 16 bytes per vertex: beyond 64 MiB
    big = rmatgen.raw_csr(n, [0, 1], [1, 2])
    g = make(big, relabel=False)
    for prog, dt in (("cc", torch.int32), ("sssp", torch.int32), ("pagerank", torch.float32)):
        with pytest.raises(VcError) as e:
            g.run_noalloc(prog, torch.empty(n, dtype=dt, device="cuda"))
        assert e.value.status == vc.ERR_INVALID_ARG and "bytes" in str(e.value)
    d = rmatgen.rmat(10, 8, seed=47, weighted=True)
    gd = make(d)
    out = torch.empty(d.n, dtype=torch.int32, device="cuda")
    for kw in (dict(schedule="blocked"), dict(options=vc.OPT_GRAPH_CAPTURE), dict(schedule="pull")):
        with pytest.raises(VcError) as e:
            gd.run_noalloc("sssp", out, source=0, **kw)
        assert e.value.status == vc.ERR_UNSUPPORTED, kw
    gd.prepare("sssp", schedule="pull")
    same("sssp", gd, source=0, schedule="pull")  # accepted once the transpose exists
