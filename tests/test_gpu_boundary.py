"""Boundary behaviour of the C ABI on the GPU.

* VC_GRAPH_SYMMETRIC with VC_GRAPH_VALIDATE: graphs that differ from their
  transpose (structure, edge multiplicity or weights) are refused with
  VC_ERR_BAD_GRAPH; symmetric ones are accepted and run.
* Captured PageRank loops stay correct when runs in other message modes come
  in between (the captured graph must never replay freed workspace).
* Hub aggregation in the push forms (LDS pre-combination of messages to the
  lowest-id, highest-degree targets) changes no result: min programs and
  fixed-point sums bit for bit with and without it, and against the oracle.
"""
import numpy as np
import pytest

import oracle
import rmatgen
from gpu_util import check_min, check_rank, run_gpu

pytestmark = pytest.mark.gpu


def upload(csr):
    import torch
    off = torch.from_numpy(np.ascontiguousarray(csr.off)).cuda()
    dst = torch.from_numpy(np.ascontiguousarray(csr.dst)).cuda()
    w = None if csr.w is None else torch.from_numpy(np.ascontiguousarray(csr.w).view(np.int32)).cuda()
    return off, dst, w


def create(csr, **kw):
    from paper_2010_01542_amd import Graph
    off, dst, w = upload(csr)
    return Graph(off, dst, w, **kw)


def symmetric_weights(csr, seed=3):
    """The same weight on u->v and v->u: a function of the unordered pair."""
    src = np.repeat(np.arange(csr.n), csr.outdeg).astype(np.uint64)
    dst = csr.dst.astype(np.uint64)
    lo, hi = np.minimum(src, dst), np.maximum(src, dst)
    return (((lo * np.uint64(2654435761) + hi * np.uint64(40503) + np.uint64(seed)) % np.uint64(255)) + 1).astype(
        np.uint32)


def test_symmetric_declaration_is_validated(device):
    from paper_2010_01542_amd import VcError, vc
    print("case symmetric validation", flush=True)
    u = rmatgen.rmat(11, 8, seed=21, directed=False)
    g = create(u, symmetric=True, validate=True)  # accepted, and runs
    check_min(u, g, "cc")
    us = rmatgen.Csr(u.n, u.m, u.off, u.dst, symmetric_weights(u))
    g = create(us, symmetric=True, validate=True)
    check_min(us, g, "sssp", source=1, schedule="pull")  # the pull form reads the CSR as its transpose
    loops = rmatgen.raw_csr(4, [0, 1, 1, 2, 3], [0, 1, 1, 3, 2], [7, 2, 2, 5, 5])  # self-loops count once each
    create(loops, symmetric=True, validate=True)
    create(rmatgen.raw_csr(3, [], []), symmetric=True, validate=True)
    bad = {
        "directed": rmatgen.rmat(11, 8, seed=22, weighted=True),
        "one reversed edge missing": rmatgen.raw_csr(3, [0, 1, 1], [1, 0, 2]),
        "multiplicity": rmatgen.raw_csr(2, [0, 0, 1], [1, 1, 0]),
        "weights": rmatgen.raw_csr(2, [0, 1], [1, 0], [3, 4]),
        "rmat weights per direction": rmatgen.from_edges(u.n, np.repeat(np.arange(u.n), u.outdeg), u.dst,
                                                         directed=False, weighted=True),
    }
    for name, c in bad.items():
        with pytest.raises(VcError) as e:
            create(c, symmetric=True, validate=True)
        assert e.value.status == vc.ERR_BAD_GRAPH, name
        create(c, symmetric=False, validate=True)  # the same CSR without the declaration is fine
        create(c, symmetric=True, validate=False)  # and the declaration is trusted without VALIDATE


def test_captured_pagerank_survives_mode_changes(device):
    """Captured binary32-accumulate, then eager fixed point (the buffers the
    capture recorded must not move), then the same captured run again; and
    the other modes interleaved the same way."""
    from paper_2010_01542_amd import vc
    print("case captured PageRank across message modes", flush=True)
    d = rmatgen.rmat(13, 16, seed=31)
    g = create(d)
    cap = vc.OPT_GRAPH_CAPTURE
    f32, f32m = vc.OPT_F32_ACCUMULATE, vc.OPT_F32_MESSAGES
    seq = [cap | f32, 0, cap | f32, f32m, cap | f32, cap, f32, cap, cap | f32m, 0, cap | f32m, cap | f32]
    first = {}
    for opt in seq:
        got = check_rank(d, g, "pagerank", T=10, options=opt)[0]
        if opt & cap and not opt & f32:  # exact sums: every replay is bit-identical
            assert np.array_equal(first.setdefault(opt, got), got), opt
    blocked = create(d)
    for opt in (cap | f32m, 0, cap | f32m, cap, f32m, cap):
        check_rank(d, blocked, "pagerank", T=6, schedule="blocked", options=opt)


@pytest.mark.parametrize("sched", ["vertex", "edge"])
@pytest.mark.parametrize("relabel", [True, False])
def test_hub_aggregation_changes_no_result(device, sched, relabel):
    from paper_2010_01542_amd import vc
    print(f"case hub aggregation schedule={sched} relabel={relabel}", flush=True)
    off_hub = vc.OPT_NO_HUB_AGGREGATION
    d = rmatgen.rmat(14, 16, seed=41, weighted=True)
    u = rmatgen.rmat(14, 16, seed=42, directed=False)
    gd, gu = create(d, relabel=relabel), create(u, relabel=relabel)
    for opt in (0, off_hub):
        check_min(d, gd, "sssp", source=0, schedule=sched, options=opt)
        check_min(u, gu, "cc", schedule=sched, options=opt)
        check_rank(d, gd, "pagerank", T=8, schedule=sched, options=opt)
        check_rank(d, gd, "pagerank", T=8, schedule=sched, options=opt | vc.OPT_F32_ACCUMULATE)
    for prog, kw in (("sssp", {"source": 0}), ("cc", {})):
        g = gd if prog == "sssp" else gu
        a, sa = run_gpu(g, prog, schedule=sched, **kw)
        b, sb = run_gpu(g, prog, schedule=sched, options=off_hub, **kw)
        assert np.array_equal(a, b) and sa.frontier.tolist() == sb.frontier.tolist()
    for opt in (0, vc.OPT_F32_MESSAGES):  # exact sums: identical with and without the table
        a = run_gpu(gd, "pagerank", T=8, schedule=sched, options=opt)[0]
        b = run_gpu(gd, "pagerank", T=8, schedule=sched, options=opt | off_hub)[0]
        assert np.array_equal(a, b)
    # every message addressed to a hub: in-star into vertex 0, and a graph
    # smaller than the table
    for c in (rmatgen.in_star(20000), rmatgen.in_star(50), rmatgen.complete_digraph(30)):
        g = create(c, relabel=relabel)
        for opt in (0, off_hub):
            check_rank(c, g, "pagerank", T=5, schedule=sched, options=opt)
            check_min(c, g, "sssp", source=1, schedule=sched, options=opt)
