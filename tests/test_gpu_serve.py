"""Request server (GPU): every request's result is the same alone and in the
mix.

* Lane tables (continuous batching of CC / SSSP): values bit-exact and
  superstep counts equal to the same request run alone with vc_run, and to
  the oracle; more requests than lanes, so lanes are retired and reseeded
  many times, and supersteps run in both the push and the pull form; a
  request stopped at its superstep cap frees its lane cleanly.
* Rank lanes and workers: PageRank / PPR equal their alone runs bit for bit
  (the default combiner sums in exact fixed point, so neither the order of
  additions nor the company of other lanes can change a result) and the
  oracle within the PageRank bars; lanes at different iteration counts
  share supersteps.
* Admission: with a budget that holds one workspace, requests still all
  complete correctly; a request whose workspace can never fit completes
  with VC_ERR_OUT_OF_MEMORY alone; a bad request is refused at submission.
"""
import numpy as np
import pytest

import oracle
import rmatgen
from gpu_util import L1_TOL, MAX_ABS_TOL, rank_errors

pytestmark = pytest.mark.gpu


def make(csr, **kw):
    from paper_2010_01542_amd import Graph
    return Graph.from_csr(csr, **kw)


def alone(csr, program, **kw):
    """Result and superstep count of the request run alone (its own graph object)."""
    import torch
    from paper_2010_01542_amd import VcError, vc
    g = make(csr, symmetric=kw.pop("symmetric", False))
    rank = program in ("pagerank", "ppr")
    out = torch.empty(csr.n, dtype=torch.float32 if rank else torch.int32, device="cuda")
    try:
        _, st = g.run(program, out, stats=True, **kw)
        status, steps = vc.OK, st.supersteps
    except VcError as e:
        status, steps = e.status, None
    vals = out.cpu().numpy()
    return (vals if rank else vals.view(np.uint32)), status, steps


def collect(srv, count):
    done = {}
    srv.drain()
    while len(done) < count:
        for c in srv.poll(timeout_ms=1000, cap=512):
            done[c.ticket] = c
    return done


@pytest.mark.parametrize("lanes", [64, 256])
def test_lanes_equal_alone_runs(device, lanes):
    import torch
    from paper_2010_01542_amd import Server, vc
    print(f"case serve lanes={lanes}", flush=True)
    d = rmatgen.rmat(11, 10, seed=5, weighted=True)
    rng = np.random.default_rng(lanes)
    sources = rng.integers(0, d.n, 3 * lanes // 2 + 7)
    deg = d.outdeg
    sources[0] = int(np.flatnonzero(deg == 0)[0])  # cannot send: ends after one superstep
    sources[1] = sources[2]
    progs = ["sssp"] * len(sources)
    for i in range(5, len(progs), 17):
        progs[i] = "cc"
    g = make(d)
    with Server(workers=1) as srv:
        gid = srv.add_graph(g, lanes=lanes)
        outs = [torch.full((d.n,), -7, dtype=torch.int32, device=device) for _ in progs]
        tickets = [srv.submit(gid, p, o, source=int(s), tag=i, route="lanes")
                   for i, (p, s, o) in enumerate(zip(progs, sources, outs))]
        done = collect(srv, len(tickets))
        info = srv.info()
    assert info["lane_requests"] == len(progs) and info["submitted"] == info["completed"] == len(progs)
    # both superstep forms ran: pushed from a broadcast list, and pulled
    assert 0 < info["lane_push_supersteps"] < info["lane_supersteps"], info
    cache = {}
    for i, (t, p, s) in enumerate(zip(tickets, progs, sources)):
        c = done[t]
        assert c.tag == i and c.status == vc.OK and 0 <= c.lane < lanes, (i, c)
        key = (p, int(s) if p == "sssp" else 0)
        if key not in cache:
            cache[key] = alone(d, p, source=key[1])
        ref, status, steps = cache[key]
        got = outs[i].cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref), (i, p, int(s), int((got != ref).sum()))
        assert status == vc.OK and c.supersteps == steps, (i, p, c.supersteps, steps)
    for p, s in list(cache)[:6]:
        o = oracle.run(p, d.n, d.off, d.dst, d.w if p == "sssp" else None, source=s)
        assert np.array_equal(cache[(p, s)][0], o.values) and cache[(p, s)][2] == o.supersteps


def test_lane_superstep_cap_frees_the_lane(device):
    import torch
    from paper_2010_01542_amd import Server, vc
    print("case serve lane cap", flush=True)
    d = rmatgen.path(200, directed=True)
    g = make(d)
    with Server(workers=1) as srv:
        gid = srv.add_graph(g, lanes=64)
        capped = torch.full((d.n,), -7, dtype=torch.int32, device=device)
        t_cap = srv.submit(gid, "sssp", capped, source=0, max_supersteps=7, route="lanes")
        outs = [torch.full((d.n,), -7, dtype=torch.int32, device=device) for _ in range(150)]
        ts = [srv.submit(gid, "sssp", o, source=i, route="lanes") for i, o in enumerate(outs)]
        done = collect(srv, 151)
    c = done[t_cap]
    ref, status, _ = alone(d, "sssp", source=0, max_supersteps=7)
    assert c.status == status == vc.ERR_NOT_CONVERGED and c.supersteps == 7 and c.lane >= 0
    assert np.array_equal(capped.cpu().numpy().view(np.uint32), ref)
    for i, (t, o) in enumerate(zip(ts, outs)):
        got = o.cpu().numpy().view(np.uint32)
        expect = np.where(np.arange(d.n) >= i, np.arange(d.n) - i, 0xFFFFFFFF).astype(np.uint32)
        assert done[t].status == vc.OK and done[t].lane >= 0 and np.array_equal(got, expect), i
        assert done[t].supersteps == d.n - i, (i, done[t].supersteps)


@pytest.mark.parametrize("route", ["auto", "lanes", "worker"])
def test_mixed_programs_on_workers_and_lanes(device, route):
    import torch
    from paper_2010_01542_amd import Server, vc
    print(f"case serve mixed programs route={route}", flush=True)
    a = rmatgen.rmat(12, 8, seed=21, weighted=True)             # lanes for its CC / SSSP
    b = rmatgen.rmat(11, 8, seed=22, directed=False)            # no lanes: everything on workers
    ga, gb = make(a), make(b, symmetric=True)
    rng = np.random.default_rng(3)
    reqs = []
    for i in range(60):
        csr, gname = (a, "a") if i % 2 == 0 else (b, "b")
        prog = ["sssp", "ppr", "pagerank", "cc", "sssp"][i % 5]
        reqs.append((csr, gname, prog, int(rng.integers(0, csr.n)), 5 + i % 7))
    with Server(workers=3) as srv:
        ids = {"a": srv.add_graph(ga, lanes=64, rank_lanes=64), "b": srv.add_graph(gb, lanes=0)}
        outs, tickets = [], []
        for csr, gname, prog, src, T in reqs:
            rank = prog in ("pagerank", "ppr")
            o = torch.full((csr.n,), -7, dtype=torch.float32 if rank else torch.int32, device=device)
            outs.append(o)
            tickets.append(srv.submit(ids[gname], prog, o, source=src, T=T, route=route))
        done = collect(srv, len(reqs))
    for (csr, gname, prog, src, T), o, t in zip(reqs, outs, tickets):
        c = done[t]
        assert c.status == vc.OK, c
        if c.lane >= 0:  # routed by expected completion time; only graph a has lane tables
            assert gname == "a" and route != "worker"
        elif route == "lanes":
            assert gname != "a"
        rank = prog in ("pagerank", "ppr")
        kw = {"T": T} if rank else {}
        ref, status, steps = alone(csr, prog, source=src, symmetric=gname == "b", **kw)
        got = o.cpu().numpy() if rank else o.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref), (gname, prog, src)
        assert c.supersteps == steps
        if rank and src % 3 == 0:
            ora = oracle.run(prog, csr.n, csr.off, csr.dst, T=T, source=src).values
            l1, mx = rank_errors(got, ora)
            assert l1 <= L1_TOL and mx <= MAX_ABS_TOL


def test_worker_views_share_the_blocked_layout(device):
    """PageRank / PPR on a graph of 2^20 vertices run in the blocked form;
    worker views share the base graph's layout, built once by whichever view
    needs it first while the others wait.  Results equal the alone runs bit
    for bit, with uint64 and with binary32 messages."""
    import torch
    from paper_2010_01542_amd import Server, vc
    print("case serve blocked layout shared by worker views (scale 20)", flush=True)
    d = rmatgen.rmat(20, 4, seed=41)
    g = make(d)
    reqs = [("ppr" if i % 3 else "pagerank", int(i * 7919) % d.n, 3 + i % 4,
             vc.OPT_F32_MESSAGES if i % 2 else 0) for i in range(12)]
    with Server(workers=4) as srv:
        gid = srv.add_graph(g)
        outs, tickets = [], []
        for prog, src, T, opt in reqs:
            o = torch.full((d.n,), -7.0, dtype=torch.float32, device=device)
            outs.append(o)
            tickets.append(srv.submit(gid, prog, o, source=src, T=T, options=opt, route="worker"))
        done = collect(srv, len(reqs))
    for (prog, src, T, opt), o, t in zip(reqs, outs, tickets):
        assert done[t].status == vc.OK, done[t]
        ref, status, steps = alone(d, prog, source=src, T=T, options=opt)
        assert np.array_equal(o.cpu().numpy(), ref), (prog, src, T, opt)
        assert done[t].supersteps == steps


def test_admission_under_a_small_budget(device):
    import torch
    from paper_2010_01542_amd import Server, VcError, vc
    print("case serve admission", flush=True)
    small = rmatgen.rmat(10, 8, seed=7)
    big = rmatgen.rmat(14, 8, seed=8)
    gs, gb = make(small), make(big)
    _, need_small = make(small).footprint("pagerank")
    _, need_big = make(big).footprint("pagerank")
    assert need_big > 2 * need_small
    budget = int(need_small * 1.5)
    with Server(workers=3, hbm_budget=budget) as srv:
        i_s, i_b = srv.add_graph(gs), srv.add_graph(gb)
        with pytest.raises(VcError) as e:  # a lane table of the big graph is over budget
            srv.add_graph(gb, lanes=64)
        assert e.value.status == vc.ERR_OUT_OF_MEMORY
        with pytest.raises(VcError):
            srv.submit(i_s, "sssp", torch.empty(small.n, dtype=torch.int32, device=device), source=small.n)
        with pytest.raises(VcError):
            srv.submit(99, "sssp", torch.empty(small.n, dtype=torch.int32, device=device))
        outs = [torch.empty(small.n, dtype=torch.float32, device=device) for _ in range(12)]
        ts = [srv.submit(i_s, "ppr", o, source=k, T=6) for k, o in enumerate(outs)]
        t_big = srv.submit(i_b, "pagerank", torch.empty(big.n, dtype=torch.float32, device=device), T=3)
        t_tail = srv.submit(i_s, "pagerank", torch.empty(small.n, dtype=torch.float32, device=device), T=2)
        done = collect(srv, len(ts) + 2)
        info = srv.info()
    assert done[t_big].status == vc.ERR_OUT_OF_MEMORY and "workspace" in done[t_big].message
    assert done[t_tail].status == vc.OK
    assert info["bytes_held"] <= budget
    for k, (t, o) in enumerate(zip(ts, outs)):
        assert done[t].status == vc.OK
        ref, _, _ = alone(small, "ppr", source=k, T=6)
        assert np.array_equal(o.cpu().numpy(), ref), k


@pytest.mark.parametrize("rank_lanes", [64, 128])
def test_rank_lanes_equal_alone_runs(device, rank_lanes):
    import torch
    from paper_2010_01542_amd import Server, vc
    print(f"case serve rank lanes={rank_lanes}", flush=True)
    d = rmatgen.rmat(11, 12, seed=9)
    rng = np.random.default_rng(rank_lanes)
    reqs = []
    for i in range(rank_lanes + 40):
        prog = "pagerank" if i % 9 == 0 else "ppr"
        reqs.append((prog, int(rng.integers(0, d.n)), int([1, 3, 7, 12, 20][i % 5]), [0.85, 0.5][i % 2]))
    reqs.append(("ppr", int(np.flatnonzero(d.outdeg == 0)[0]), 6, 0.85))  # a source without out-edges
    g = make(d)
    with Server(workers=1) as srv:
        gid = srv.add_graph(g, rank_lanes=rank_lanes)
        outs = [torch.full((d.n,), -1.0, dtype=torch.float32, device=device) for _ in reqs]
        ts = [srv.submit(gid, p, o, source=src, T=T, damping=dd, route="lanes")
              for (p, src, T, dd), o in zip(reqs, outs)]
        t0 = srv.submit(gid, "ppr", torch.empty(d.n, dtype=torch.float32, device=device), source=3, T=0)
        t32 = srv.submit(gid, "ppr", torch.empty(d.n, dtype=torch.float32, device=device), source=3, T=4,
                         options=vc.OPT_F32_ACCUMULATE)
        done = collect(srv, len(ts) + 2)
        info = srv.info()
    assert done[t0].status == vc.OK and done[t0].lane == -1  # T = 0 and binary32 sums run on workers
    assert done[t32].status == vc.OK and done[t32].lane == -1
    assert info["rank_requests"] == len(reqs)
    for k, ((p, src, T, dd), o, t) in enumerate(zip(reqs, outs, ts)):
        c = done[t]
        assert c.status == vc.OK and 0 <= c.lane < rank_lanes and c.supersteps == T + 1, (k, c)
        ref, status, steps = alone(d, p, source=src, T=T, damping=dd)
        got = o.cpu().numpy()
        assert np.array_equal(got, ref), (k, p, src, T, float(np.abs(got - ref).max()))
        if k < 6:
            ora = oracle.run(p, d.n, d.off, d.dst, T=T, damping=dd, source=src).values
            l1, mx = rank_errors(got, ora)
            assert l1 <= L1_TOL and mx <= MAX_ABS_TOL, (k, l1, mx)
