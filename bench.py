#!/usr/bin/env python3
"""Benchmark of the Pregel superstep path on one MI355X.

A step is one pass of the whole hot path over one synthetic graph already
resident in HBM:
  sssp-s26 (default): SSSP from vertex 0 to quiescence + PageRank T=20 on a
            directed R-MAT scale-26 graph, edge factor 16 (~1.06 B edges),
            int64 offsets, uint32 weights in [1, 255];
  cc-s22:   hash-min CC to quiescence on an undirected R-MAT scale-22 graph;
  pr-s16:   PageRank T=10 on a directed R-MAT scale-16 graph.
value = traversed edges (sum of E_s over all supersteps of the step) per
second, in GTEPS.  The roofline object reports the dominant kernel (the
broadcast+combine of the superstep) against the 8 TB/s HBM peak, from HIP
events recorded on the run's stream around every launch of that kernel.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info():
    info = {"nproc": os.cpu_count()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name"):
                info["cpu"] = line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        with open("/proc/meminfo") as f:
            info["mem_gib"] = round(int(f.readline().split()[1]) / 2**20, 1)
    except Exception:
        pass
    return info


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("paper_2010_01542_amd/csrc/vc_pull.hip", "paper_2010_01542_amd/csrc/vc_device.h"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch of the PageRank pull kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs, or None when the kernel source
    changed since they were taken (or none exist for this workload)."""
    path = os.path.join(ROOT, "profiles", "pr_pull_s26_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except OSError:
        return None
    if rec.get("workload") != workload or rec.get("source_hash") != kernel_source_hash():
        return None
    return int(rec["traffic_bytes_per_launch"])


def pr_scatter_bytes(n, m, off_bytes):
    """Algorithmic bytes of one PageRank broadcast+combine launch:
    offsets (N+1) + per-vertex message (4N) + targets (4M) + 4-byte mailbox
    read-modify-write per message (8M)."""
    return (n + 1) * off_bytes + 4 * n + 12 * m


def batch_members(count, seed):
    """Seeded batch: scales uniform on [10, 16], edge factor uniform on [8, 32],
    each graph SSSP (directed, uint32 weights, source 0) or hash-min CC
    (symmetrised) with probability 1/2."""
    import rmatgen
    rng = np.random.default_rng(seed)
    csrs, queries = [], []
    for j in range(count):
        scale, ef = int(rng.integers(10, 17)), int(rng.integers(8, 33))
        if rng.random() < 0.5:
            csrs.append(rmatgen.rmat(scale, ef, seed=seed * 7919 + j, weighted=True))
            queries.append(("sssp", 0))
        else:
            csrs.append(rmatgen.rmat(scale, ef, seed=seed * 7919 + j, directed=False))
            queries.append(("cc", 0))
    return csrs, queries


def bench_batch(args, dev):
    """Plain path (one vc_run per graph, one after another) vs one batched run
    over the union; both relax the same messages superstep by superstep."""
    import torch
    import rmatgen
    from paper_2010_01542_amd import Batch, Graph
    t = time.time()
    csrs, queries = batch_members(args.members, rmatgen.BASE_SEED + 3)
    n_tot, m_tot = sum(c.n for c in csrs), sum(c.m for c in csrs)
    log(f"generated {len(csrs)} graphs, {n_tot} vertices, {m_tot} edges in {time.time() - t:.1f}s")
    graphs = [Graph.from_csr(c, device=dev) for c in csrs]
    outs = [torch.empty(c.n, dtype=torch.int32, device=dev) for c in csrs]
    for g, o, (prog, src) in zip(graphs, outs, queries):  # warm-up: workspaces, transposes
        g.run(prog, o, source=src)
    torch.cuda.synchronize()
    lat, edges_plain = [], 0
    t0 = time.perf_counter()
    for g, o, (prog, src) in zip(graphs, outs, queries):
        a = time.perf_counter()
        _, st = g.run(prog, o, source=src, stats=True)
        lat.append(time.perf_counter() - a)
        edges_plain += st.edges_relaxed
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    # the same plain runs with each graph's superstep loop captured as a HIP graph
    from paper_2010_01542_amd import vc
    cap = vc.OPT_GRAPH_CAPTURE
    for g, o, (prog, src) in zip(graphs, outs, queries):
        g.run(prog, o, source=src, options=cap)
    torch.cuda.synchronize()
    lat_cap = []
    t0 = time.perf_counter()
    for g, o, (prog, src) in zip(graphs, outs, queries):
        a = time.perf_counter()
        g.run(prog, o, source=src, options=cap)
        lat_cap.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    plain_cap_s = time.perf_counter() - t0
    del graphs
    torch.cuda.empty_cache()
    b = Batch(csrs, queries, device=dev)
    tuned = b.autotune()
    log(f"batch autotune picked {tuned}")
    out = torch.empty(b.n, dtype=torch.int32, device=dev)
    for _ in range(args.warmup):
        b.run(out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = b.run(out, stats=True)
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - t0) / args.steps
    assert st.edges_relaxed == edges_plain, (st.edges_relaxed, edges_plain)
    lat_ms = np.array(lat) * 1e3
    return {
        "metric": "GTEPS & HBM GB/s vs peak per superstep; batched/served p50/p99 vs plain",
        "value": round(edges_plain / batch_s / 1e9, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(batch_s * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic R-MAT (seeded)",
        "config": {"workload": f"batch-{len(csrs)}", "graphs": len(csrs), "vertices": n_tot, "edges": m_tot,
                   "queries": {"sssp": sum(q[0] == "sssp" for q in queries),
                               "cc": sum(q[0] == "cc" for q in queries)}},
        "batched": {"ms": round(batch_s * 1e3, 3), "gteps": round(edges_plain / batch_s / 1e9, 3),
                    "queries_per_s": round(len(csrs) / batch_s, 1), "supersteps": st.supersteps},
        "plain": {"ms": round(plain_s * 1e3, 3), "gteps": round(edges_plain / plain_s / 1e9, 3),
                  "queries_per_s": round(len(csrs) / plain_s, 1),
                  "latency_ms_p50": round(float(np.percentile(lat_ms, 50)), 3),
                  "latency_ms_p99": round(float(np.percentile(lat_ms, 99)), 3)},
        "plain_captured": {"ms": round(plain_cap_s * 1e3, 3), "queries_per_s": round(len(csrs) / plain_cap_s, 1),
                           "latency_ms_p50": round(float(np.percentile(np.array(lat_cap) * 1e3, 50)), 3),
                           "latency_ms_p99": round(float(np.percentile(np.array(lat_cap) * 1e3, 99)), 3)},
        "batch_autotuned": tuned,
        "speedup_vs_plain": round(plain_s / batch_s, 2),
        "edges_relaxed": int(edges_plain),
    }


def bench_multi(args, dev):
    """256 SSSP sources on the directed weighted R-MAT scale-22 graph: one
    plain vc_run per source vs one many-source run."""
    import torch
    import rmatgen
    from paper_2010_01542_amd import Graph
    scale = args.scale or 22
    csr = rmatgen.workload("sssp-s26", scale=scale, threads=args.gen_threads)
    deg = csr.outdeg
    rng = np.random.default_rng(rmatgen.BASE_SEED + 4)
    sources = rng.choice(np.flatnonzero(deg > 0), size=args.sources, replace=False).astype(np.uint32)
    g = Graph.from_csr(csr, device=dev)
    out1 = torch.empty(csr.n, dtype=torch.int32, device=dev)
    g.run("sssp", out1, source=int(sources[0]))
    torch.cuda.synchronize()
    lat, edges_plain = [], 0
    t0 = time.perf_counter()
    for s in sources:
        a = time.perf_counter()
        _, st = g.run("sssp", out1, source=int(s), stats=True)
        lat.append(time.perf_counter() - a)
        edges_plain += st.edges_relaxed
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    outk = torch.empty((csr.n, len(sources)), dtype=torch.int32, device=dev)
    for _ in range(args.warmup):
        g.run_multi_source(sources, outk)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, st = g.run_multi_source(sources, outk, stats=True, timing=True)
    torch.cuda.synchronize()
    multi_s = (time.perf_counter() - t0) / args.steps
    # spot check: the last plain run's source column is identical
    assert torch.equal(outk[:, -1].contiguous(), out1), "many-source column differs from the plain run"
    lat_ms = np.array(lat) * 1e3
    return {
        "metric": "GTEPS & HBM GB/s vs peak per superstep; batched/served p50/p99 vs plain",
        "value": round(edges_plain / multi_s / 1e9, 3), "unit": "GTEPS (plain-equivalent messages)", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(multi_s * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic R-MAT (seeded)",
        "config": {"workload": f"multi-source-{len(sources)}@{csr.name}", "vertices": csr.n, "edges": csr.m,
                   "sources": len(sources)},
        "batched": {"ms": round(multi_s * 1e3, 3), "queries_per_s": round(len(sources) / multi_s, 1),
                    "supersteps": st.supersteps, "superstep_ms": [round(float(x), 3) for x in st.step_ms]},
        "plain": {"ms": round(plain_s * 1e3, 3), "queries_per_s": round(len(sources) / plain_s, 1),
                  "gteps": round(edges_plain / plain_s / 1e9, 3),
                  "latency_ms_p50": round(float(np.percentile(lat_ms, 50)), 3),
                  "latency_ms_p99": round(float(np.percentile(lat_ms, 99)), 3)},
        "speedup_vs_plain": round(plain_s / multi_s, 2),
    }


def bench_combine(args, dev):
    """One superstep of message passing on the directed R-MAT graph (scale 24
    by default) with each generic combiner (flag + compare-and-swap; every
    vertex active, so the pull form runs), against the native-atomic push
    superstep of PageRank (uint64 atomic add per message) on the same graph."""
    import torch
    import rmatgen
    from paper_2010_01542_amd import Graph
    from paper_2010_01542_amd.vc import COMBINERS
    scale = args.scale or 24
    csr = rmatgen.workload("sssp-s26", scale=scale, threads=args.gen_threads)
    g = Graph.from_csr(csr, device=dev)
    rng = np.random.default_rng(rmatgen.BASE_SEED + 7)
    n, m = csr.n, csr.m
    words = {"sum_u64": rng.integers(0, 2**62, n, dtype=np.uint64),
             "prod_u64": rng.integers(0, 2**62, n, dtype=np.uint64) | np.uint64(1),
             "max_f64": rng.standard_normal(n).view(np.uint64),
             "minarg": ((rng.permutation(n).astype(np.uint64) << np.uint64(32)) |
                        rng.integers(0, 1000, n).astype(np.float32).view(np.uint32).astype(np.uint64)),
             "sum_f64": rng.standard_normal(n).view(np.uint64)}
    box = torch.empty(n, dtype=torch.int64, device=dev)
    has = torch.empty(n, dtype=torch.int32, device=dev)
    res = {}
    for op in COMBINERS:
        msg = torch.from_numpy(words[op].view(np.int64)).to(dev)
        for _ in range(args.warmup):
            g.combine(op, msg, None, box, has)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            g.combine(op, msg, None, box, has)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        res[op] = {"ms": round(dt * 1e3, 3), "gteps": round(m / dt / 1e9, 2)}
        log(f"combine {op}: {dt * 1e3:.2f} ms")
    out = torch.empty(n, dtype=torch.float32, device=dev)
    g.run("pagerank", out, T=1, schedule="edge")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.run("pagerank", out, T=1, schedule="edge")
    torch.cuda.synchronize()
    native = (time.perf_counter() - t0) / args.steps
    worst = max(v["ms"] for v in res.values())
    # pull form: per in-edge the source id and the sender's message; per
    # receiver its transpose offset, message and flag written once
    alg = 12 * m + 12 * n + (n + 1) * 8
    return {
        "metric": "messages combined per second with combiners without native atomics",
        "value": round(m / (worst / 1e3) / 1e9, 2), "unit": "GTEPS (slowest combiner)", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": worst, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64/f64", "data": "synthetic R-MAT (seeded)",
        "config": {"workload": f"combine@{csr.name}", "vertices": n, "edges": m},
        "combiners": res,
        "native_atomic_pagerank_push_superstep": {"ms": round(native * 1e3, 3), "gteps": round(m / native / 1e9, 2)},
        "roofline": {"bound": "hbm", "achieved": round(alg / (worst / 1e3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(alg / (worst / 1e3) / 1e9 / HBM_PEAK_GBS, 4), "traffic": None},
    }


SERVE_GRAPHS = (  # name, scale, directed, weighted, lanes, share of SSSP / PPR traffic, rank lanes
    ("s18", 18, True, True, 256, 0.50, 256),
    ("s22", 22, True, True, 256, 0.35, 128),
    ("s24", 24, True, True, 256, 0.15, 64),
)
SERVE_CC = ("cc-s20", 20, False, False, 64)


def serve_requests(count, graphs, seed):
    """Seeded request stream: 70% SSSP, 20% PPR (T = 20), 10% CC; SSSP and PPR
    pick a graph by its share and a uniform source with out-edges; CC runs on
    the symmetrised graph."""
    rng = np.random.default_rng(seed)
    names = [g[0] for g in SERVE_GRAPHS]
    share = np.array([g[5] for g in SERVE_GRAPHS])
    senders = {k: np.flatnonzero(c.outdeg > 0) for k, c in graphs.items()}
    reqs = []
    for _ in range(count):
        u = rng.random()
        if u < 0.1:
            reqs.append((SERVE_CC[0], "cc", 0))
            continue
        name = names[int(rng.choice(len(names), p=share))]
        src = int(rng.choice(senders[name]))
        reqs.append((name, "sssp" if u < 0.8 else "ppr", src))
    return reqs


def bench_serve(args, dev):
    """Request serving on resident graphs.  Baseline: every request run alone
    with vc_run, one after another (first-come-first-served, one stream).
    Server: lane tables (continuous batching) and worker threads, CC / SSSP
    routed between them by expected completion time, PPR on the workers.  Reports saturation throughput (all requests queued at once) and the
    latency of an open-loop Poisson arrival stream at 80% of the baseline's
    capacity, the baseline's latencies simulated from its measured service
    times on the same arrival times."""
    import torch
    import rmatgen
    from paper_2010_01542_amd import Graph, Server, vc
    t = time.time()
    csrs = {}
    for name, scale, directed, weighted, _, _, _ in SERVE_GRAPHS:
        csrs[name] = rmatgen.rmat(scale, 16, seed=rmatgen.BASE_SEED + scale, directed=directed, weighted=weighted,
                                  threads=args.gen_threads)
    name, scale, directed, weighted, _ = SERVE_CC
    csrs[name] = rmatgen.rmat(scale, 16, seed=rmatgen.BASE_SEED + 100 + scale, directed=directed,
                              weighted=weighted, threads=args.gen_threads)
    log(f"generated serving graphs in {time.time() - t:.1f}s: " +
        ", ".join(f"{k} n={c.n} m={c.m}" for k, c in csrs.items()))
    graphs = {k: Graph.from_csr(c, device=dev, symmetric=(k == SERVE_CC[0])) for k, c in csrs.items()}
    reqs = serve_requests(args.requests, csrs, rmatgen.BASE_SEED + 5)
    lanes_of = {x[0]: x[4] for x in SERVE_GRAPHS}
    lanes_of[SERVE_CC[0]] = SERVE_CC[4]
    rank_lanes_of = {x[0]: x[6] for x in SERVE_GRAPHS}
    rank_lanes_of[SERVE_CC[0]] = 0
    pool = {}

    def out_for(i, name, prog):
        key = (name, prog == "ppr", i)
        if key not in pool:
            pool[key] = torch.empty(csrs[name].n, dtype=torch.float32 if prog == "ppr" else torch.int32, device=dev)
        return pool[key]

    # baseline: each request alone, in order (warm-up: one of each kind first)
    for name, prog, src in {(r[0], r[1]): r for r in reqs}.values():
        graphs[name].run(prog, out_for(0, name, prog), source=src, T=20)
    torch.cuda.synchronize()
    service = np.zeros(len(reqs))
    t0 = time.perf_counter()
    for i, (name, prog, src) in enumerate(reqs):
        a = time.perf_counter()
        graphs[name].run(prog, out_for(0, name, prog), source=src, T=20)
        service[i] = time.perf_counter() - a
    base_s = time.perf_counter() - t0
    log(f"sequential: {len(reqs)} requests in {base_s:.2f}s")
    checks = [i for i in range(len(reqs)) if reqs[i][1] != "ppr"][:8]
    ref = {}
    for i in checks:
        name, prog, src = reqs[i]
        ref[i] = graphs[name].run(prog, source=src)[0].cpu()

    def run_server(arrivals):
        """Submits request i at arrivals[i] (seconds from start); returns the
        makespan and per-request latencies (submit -> result complete)."""
        srv = Server(workers=args.workers)
        ids = {k: srv.add_graph(g, lanes=lanes_of[k], rank_lanes=rank_lanes_of[k]) for k, g in graphs.items()}
        outs = [out_for(i, name, prog) for i, (name, prog, _) in enumerate(reqs)]
        lat = np.zeros(len(reqs))
        lanes_used = 0
        tick = {}
        t_start = time.perf_counter()
        got = 0
        for i, (name, prog, src) in enumerate(reqs):
            wait = arrivals[i] - (time.perf_counter() - t_start)
            while wait > 0:
                for c in srv.poll(timeout_ms=max(1, int(wait * 1e3)), cap=1024):
                    lat[tick[c.ticket]] = c.latency_ms
                    lanes_used += c.lane >= 0
                    got += 1
                    assert c.status == vc.OK, c.message
                wait = arrivals[i] - (time.perf_counter() - t_start)
            tick[srv.submit(ids[name], prog, outs[i], source=src, T=20)] = i
        while got < len(reqs):
            for c in srv.poll(timeout_ms=1000, cap=1024):
                lat[tick[c.ticket]] = c.latency_ms
                lanes_used += c.lane >= 0
                got += 1
                assert c.status == vc.OK, c.message
        span = time.perf_counter() - t_start
        info = srv.info()
        srv.close()
        for i in checks:
            assert torch.equal(outs[i].cpu(), ref[i]), f"served request {i} differs from its alone run"
        return span, lat, info, lanes_used

    span, lat_sat, info, lanes_used = run_server(np.zeros(len(reqs)))
    log(f"server, all queued: {len(reqs)} requests in {span:.2f}s; {info}")
    rate = 0.8 * len(reqs) / base_s
    gaps = np.random.default_rng(rmatgen.BASE_SEED + 6).exponential(1.0 / rate, len(reqs))
    arrivals = np.cumsum(gaps) - gaps[0]
    span_open, lat_open, info_open, lanes_open = run_server(arrivals)
    # the baseline on the same arrivals: one FIFO server with the measured service times
    fin, lat_base = 0.0, np.zeros(len(reqs))
    for i in range(len(reqs)):
        fin = max(fin, arrivals[i]) + service[i]
        lat_base[i] = (fin - arrivals[i]) * 1e3
    kinds = {}
    for (name, prog, _), s in zip(reqs, service):
        kinds.setdefault(f"{prog}@{name}", []).append(s * 1e3)

    def pct(a, q):
        return round(float(np.percentile(a, q)), 3)

    def by_kind(lat):
        out = {}
        for i, (name, prog, _) in enumerate(reqs):
            out.setdefault(f"{prog}@{name}", []).append(lat[i])
        return {k: [pct(v, 50), pct(v, 99)] for k, v in sorted(out.items())}

    return {
        "metric": "served requests/s (70% SSSP, 20% PPR T=20, 10% CC on resident R-MAT graphs)",
        "value": round(len(reqs) / span, 2), "unit": "requests/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(span * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32+f32", "data": "synthetic R-MAT (seeded)",
        "config": {"workload": f"serve-{len(reqs)}", "graphs": {k: [c.n, c.m] for k, c in csrs.items()},
                   "lanes": lanes_of, "rank_lanes": rank_lanes_of, "workers": args.workers,
                   "hw_queues": args.hw_queues},
        "sequential": {"requests_per_s": round(len(reqs) / base_s, 2),
                       "service_ms_mean": {k: round(float(np.mean(v)), 3) for k, v in kinds.items()}},
        "speedup_vs_sequential": round(base_s / span, 2),
        "saturated": {"latency_ms_p50": pct(lat_sat, 50), "latency_ms_p99": pct(lat_sat, 99),
                      "p50_p99_by_kind": by_kind(lat_sat),
                      "lane_requests": lanes_used, "lane_supersteps": info["lane_supersteps"],
                      "rank_supersteps": info["rank_supersteps"]},
        "open_loop": {"arrival_rate_per_s": round(rate, 2), "latency_ms_p50": pct(lat_open, 50),
                      "latency_ms_p99": pct(lat_open, 99), "sequential_latency_ms_p50": pct(lat_base, 50),
                      "sequential_latency_ms_p99": pct(lat_base, 99), "makespan_s": round(span_open, 3),
                      "lane_requests": lanes_open, "lane_supersteps": info_open["lane_supersteps"],
                      "rank_supersteps": info_open["rank_supersteps"],
                      "p50_p99_by_kind": by_kind(lat_open), "sequential_p50_p99_by_kind": by_kind(lat_base)},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sssp-s26", choices=["sssp-s26", "cc-s22", "pr-s16", "batch", "multi", "serve", "combine"])
    ap.add_argument("--sources", type=int, default=256, help="multi workload: SSSP sources")
    ap.add_argument("--members", type=int, default=1024, help="batch workload: number of graphs")
    ap.add_argument("--requests", type=int, default=600, help="serve workload: number of requests")
    ap.add_argument("--workers", type=int, default=4, help="serve workload: worker threads")
    ap.add_argument("--hw-queues", type=int, default=None,
                    help="serve workload: hardware queues of the process (GPU_MAX_HW_QUEUES, at most 32); "
                         "lane tables, rank tables and workers each use their own stream")
    ap.add_argument("--scale", type=int, default=None, help="override the graph scale (same shape)")
    ap.add_argument("--schedule", default="auto", choices=["auto", "vertex", "edge", "pull"])
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--f32-accumulate", action="store_true", help="binary32 PageRank combiner (float atomics)")
    ap.add_argument("--gen-threads", type=int, default=16)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one 1 GiB device-to-device copy first (reference for traffic counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(libvc runs on one GPU; sharding across GPUs is not implemented).", file=sys.stderr)
        sys.exit(2)

    if args.hw_queues is None and args.workload == "serve":
        args.hw_queues = 16  # one per lane table, rank table and worker stream
    if args.hw_queues:
        if not 1 <= args.hw_queues <= 32:
            sys.exit("--hw-queues must be in 1..32")
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)  # read when the HIP runtime starts, below

    import torch
    import rmatgen
    from paper_2010_01542_amd import Graph

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.workload == "batch":
        print(json.dumps(bench_batch(args, dev)), flush=True)
        return
    if args.workload == "multi":
        print(json.dumps(bench_multi(args, dev)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args, dev)), flush=True)
        return
    if args.workload == "combine":
        print(json.dumps(bench_combine(args, dev)), flush=True)
        return
    t = time.time()
    csr = rmatgen.workload(args.workload, scale=args.scale, threads=args.gen_threads)
    log(f"generated {csr.name}: n={csr.n} m={csr.m} in {time.time() - t:.1f}s")
    t = time.time()
    g = Graph.from_csr(csr, device=dev)
    log(f"uploaded in {time.time() - t:.1f}s")
    off_bytes = csr.off.dtype.itemsize
    n, m = csr.n, csr.m
    from paper_2010_01542_amd import vc
    kw = dict(schedule=args.schedule, tile=args.tile, options=vc.OPT_F32_ACCUMULATE if args.f32_accumulate else 0)

    if args.workload == "sssp-s26":
        jobs = [("sssp", dict(source=0)), ("pagerank", dict(T=20))]
        dominant = "pagerank"
    elif args.workload == "cc-s22":
        jobs = [("cc", {})]
        dominant = "cc"
    else:
        jobs = [("pagerank", dict(T=10))]
        dominant = "pagerank"

    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del a, b

    out_f = torch.empty(n, dtype=torch.float32, device=dev)
    out_u = torch.empty(n, dtype=torch.int32, device=dev)

    def step(timing):
        res = {}
        for prog, pk in jobs:
            out = out_f if prog in ("pagerank", "ppr") else out_u
            _, st = g.run(prog, out, stats=True, timing=timing, **pk, **kw)
            res[prog] = st
        return res

    for i in range(args.warmup):
        step(False)
        log(f"warmup {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    records = []
    for i in range(args.steps):
        records.append(step(True))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} steps in {elapsed:.3f}s")

    edges_per_step = sum(st.edges_relaxed for st in records[0].values())
    ms_per_step = 1e3 * elapsed / args.steps
    gteps = edges_per_step / (elapsed / args.steps) / 1e9

    detail = {}
    for prog, st in records[0].items():
        scat = np.concatenate([r[prog].scatter_ms for r in records]).reshape(len(records), -1)
        steps_ms = np.concatenate([r[prog].step_ms for r in records]).reshape(len(records), -1)
        runs_ms = [r[prog].elapsed_ms for r in records]
        detail[prog] = {
            "supersteps": st.supersteps,
            "edges": int(st.edges_relaxed),
            "run_ms_median": float(np.median(runs_ms)),
            "frontier": st.frontier.tolist(),
            "edges_per_superstep": st.edges.tolist(),
            "scatter_ms_median": np.median(scat, axis=0).round(4).tolist(),
            "superstep_ms_median": np.median(steps_ms, axis=0).round(4).tolist(),
            "schedule": st.schedule.tolist(),
        }

    roofline = None
    if dominant == "pagerank":
        scat = np.concatenate([r["pagerank"].scatter_ms[:-1] for r in records])
        avg_ms = float(scat.mean())
        bytes_launch = pr_scatter_bytes(n, m, off_bytes)
        achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
        sched = records[0]["pagerank"].schedule[0]
        kname = {1: "k_pr_scatter_vertex", 2: "k_pr_scatter_mp", 3: "k_pr_pull"}.get(int(sched), "?")
        traffic = measured_traffic(csr.name) if (kname == "k_pr_pull" and not args.f32_accumulate) else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                    "kernel": f"{kname} (PageRank broadcast+combine)", "launches": int(scat.size),
                    "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": int(bytes_launch),
                    "gteps_per_launch": round(m / (avg_ms * 1e-3) / 1e9, 2)}

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        sample_T = 1
        t = time.perf_counter()
        oracle.run_csr("pagerank", csr, T=sample_T)
        dt = time.perf_counter() - t
        cpu = {"value": round(sample_T * m / dt / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"oracle PageRank, {sample_T} broadcast+combine superstep(s) over the full graph "
                         f"({sample_T * m} messages), single thread, {dt:.1f}s"}
        log(f"cpu baseline: {cpu['value']} GTEPS in {dt:.1f}s")

    res = {
        "metric": "GTEPS & HBM GB/s vs peak per superstep; batched/served p50/p99 vs plain",
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+u32",
        "data": "synthetic R-MAT (seeded)",
        "config": {"workload": csr.name, "vertices": n, "edges": m,
                   "offsets": "int64" if off_bytes == 8 else "int32",
                   "steps": " + ".join(f"{p}{'(T=%d)' % k['T'] if 'T' in k else ''}" for p, k in jobs),
                   "schedule": args.schedule, "tile": args.tile or "default"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": detail,
        "host": host_info(),
        "device": torch.cuda.get_device_name(0),
        "python": platform.python_version(),
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
