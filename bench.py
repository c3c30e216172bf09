#!/usr/bin/env python3
"""Benchmark of the Pregel superstep path on one MI355X.

A step is one pass of the whole hot path over one synthetic graph already
resident in HBM:
  sssp-s26 (default): SSSP from vertex 0 to quiescence + PageRank T=20 on a
            directed R-MAT scale-26 graph, edge factor 16 (~1.06 B edges),
            int64 offsets, uint32 weights in [1, 255];
  cc-s22:   hash-min CC to quiescence on an undirected R-MAT scale-22 graph;
  pr-s16:   PageRank T=10 on a directed R-MAT scale-16 graph.
PageRank sums are exact (uint64 fixed point); its messages are binary32 by
default (--messages u64 for uint64 messages, --f32-accumulate for float
atomics instead).  value = traversed edges (sum of E_s over all supersteps of
the step) per second, in GTEPS.  The roofline object reports the dominant kernel (the
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


KERNEL_SOURCES = {"pull": ("vc_pull.hip", "vc_device.h"), "blocked": ("vc_blocked.hip", "vc_device.h")}


def kernel_source_hash(form):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[form]:
        with open(os.path.join(ROOT, "paper_2010_01542_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload, form, options):
    """HBM bytes per PageRank broadcast+combine of the pull or blocked form
    from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE runs, or None when
    the kernel source changed since they were taken (or none exist for this
    workload and these options)."""
    path = os.path.join(ROOT, "profiles", f"pr_{form}_s26_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except OSError:
        return None
    if (rec.get("workload") != workload or rec.get("source_hash") != kernel_source_hash(form)
            or rec.get("options", 0) != options):
        return None
    return int(rec["traffic_bytes_per_launch"])


def pr_scatter_bytes(n, m, off_bytes):
    """Algorithmic bytes of one PageRank broadcast+combine launch:
    offsets (N+1) + per-vertex message (4N) + targets (4M) + 4-byte mailbox
    read-modify-write per message (8M)."""
    return (n + 1) * off_bytes + 4 * n + 12 * m


def pr_superstep_bytes(n, m, off_bytes):
    """Algorithmic bytes of a whole PageRank superstep: the broadcast+combine
    plus the vertex update's 4-byte rank write per vertex."""
    return pr_scatter_bytes(n, m, off_bytes) + 4 * n


def min_superstep_bytes(n, off_bytes, weighted, frontier, edges, receivers, dense0):
    """Algorithmic bytes of every CC / SSSP superstep s (the method's nominal
    traffic): per sender its id, value and two offsets, per message its
    target, weight and a 4-byte mailbox read-modify-write, per receiver its
    mailbox, value and flag, per vertex activated next its id and degree.
    A dense superstep 0 (CC: every vertex sends) reads values and offsets by
    vertex id instead: N (4 + o).  frontier / edges / receivers: |F_s|, E_s,
    |R_s| per superstep (|F_{s+1}| is the next superstep's frontier)."""
    w = 4 if weighted else 0
    out = []
    for s in range(len(frontier)):
        nxt = frontier[s + 1] if s + 1 < len(frontier) else 0
        senders = n * (4 + off_bytes) if (s == 0 and dense0) else frontier[s] * (8 + 2 * off_bytes)
        out.append(int(senders + edges[s] * (12 + w) + receivers[s] * 12 + nxt * 8))
    return out


def cpu_pool_cores():
    """Host cores a pool of oracle runs may use: the ones this process may
    run on, at most 16 (one GPU's share of the machine's CPUs)."""
    return max(1, min(16, len(os.sched_getaffinity(0))))


def cpu_pool_baseline(tasks, what, expect=None):
    """CPU throughput baseline for many independent queries: the oracle (a
    single-threaded C engine that releases the interpreter lock while it
    runs) on every task, `cores` at a time on a thread pool.  tasks: (program,
    csr, source, T) tuples.  Reports messages and queries per second of wall
    time.  expect (optional): expect(i) gives the device's values for task i,
    which must equal the oracle's (CC labels, SSSP distances), or None where
    no such check applies; "equal_device" counts the equal ones."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    cores = cpu_pool_cores()

    def one(i):
        prog, c, src, T = tasks[i]
        r = oracle.run(prog, c.n, c.off, c.dst, c.w if prog == "sssp" else None, source=src, T=T)
        dev_vals = None if expect is None else expect(i)
        ok = dev_vals is None or bool(np.array_equal(dev_vals, r.values))
        return int(r.messages.sum()), ok, dev_vals is not None

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as pool:
        res = list(pool.map(one, range(len(tasks))))
    wall = time.perf_counter() - t0
    msgs = sum(r[0] for r in res)
    equal = sum(r[1] and r[2] for r in res)
    checked = sum(r[2] for r in res)
    log(f"cpu pool baseline ({what}): {len(tasks)} queries, {msgs} messages in {wall:.1f}s on {cores} threads")
    return {"value": round(msgs / wall / 1e9, 4), "unit": "GTEPS", "cores": cores, "kind": "oracle",
            "queries_per_s": round(len(tasks) / wall, 2),
            "equal_device": None if expect is None else f"{equal}/{checked}",
            "sample": f"{what}: {len(tasks)} independent oracle runs ({msgs} messages) on a pool of {cores} "
                      f"threads, one query per thread at a time, {wall:.1f}s wall"}


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
    out = torch.empty(b.n, dtype=torch.int32, device=dev)
    # the host-driven and the captured superstep loop (forms switched on the
    # device), AUTO's defaults, before the autotuner picks its setting
    forms = {}
    for name, opt in (("eager", 0), ("captured", vc.OPT_GRAPH_CAPTURE)):
        for _ in range(max(1, args.warmup)):
            b.run(out, options=opt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.run(out, options=opt)
        torch.cuda.synchronize()
        forms[name] = round((time.perf_counter() - t0) / args.steps * 1e3, 3)
    log(f"batch loop forms (ms per batch): {forms}")
    tuned = b.autotune()
    log(f"batch autotune picked {tuned}")
    for _ in range(args.warmup):
        b.run(out)
    torch.cuda.synchronize()
    blat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        _, st = b.run(out, stats=True)
        blat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    batch_s = (time.perf_counter() - t0) / args.steps
    assert st.edges_relaxed == edges_plain, (st.edges_relaxed, edges_plain)
    # every member's batched result against its plain run (outs hold the plain runs' results)
    same = sum(bool(np.array_equal(x, o.cpu().numpy().view(np.uint32))) for x, o in zip(b.split(out), outs))
    if same != len(csrs):
        raise SystemExit(f"batched results differ from the plain runs for {len(csrs) - same} members")
    blat_ms = np.array(blat) * 1e3
    lat_ms = np.array(lat) * 1e3
    cpu = None if args.no_cpu_baseline else cpu_pool_baseline(
        [(prog, c, src, 10) for c, (prog, src) in zip(csrs, queries)], "every member of the batch")
    return {
        "metric": "GTEPS & HBM GB/s vs peak per superstep; batched/served p50/p99 vs plain",
        "value": round(edges_plain / batch_s / 1e9, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(batch_s * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic R-MAT (seeded)",
        "config": {"workload": f"batch-{len(csrs)}", "graphs": len(csrs), "vertices": n_tot, "edges": m_tot,
                   "queries": {"sssp": sum(q[0] == "sssp" for q in queries),
                               "cc": sum(q[0] == "cc" for q in queries)}},
        "batched": {"ms": round(batch_s * 1e3, 3), "gteps": round(edges_plain / batch_s / 1e9, 3),
                    "queries_per_s": round(len(csrs) / batch_s, 1), "supersteps": st.supersteps,
                    "latency_ms_p50": round(float(np.percentile(blat_ms, 50)), 3),
                    "latency_ms_p99": round(float(np.percentile(blat_ms, 99)), 3),
                    "members_equal_plain": f"{same}/{len(csrs)}"},
        "batched_loop_ms": forms,
        "plain": {"ms": round(plain_s * 1e3, 3), "gteps": round(edges_plain / plain_s / 1e9, 3),
                  "queries_per_s": round(len(csrs) / plain_s, 1),
                  "latency_ms_p50": round(float(np.percentile(lat_ms, 50)), 3),
                  "latency_ms_p99": round(float(np.percentile(lat_ms, 99)), 3)},
        "plain_captured": {"ms": round(plain_cap_s * 1e3, 3), "queries_per_s": round(len(csrs) / plain_cap_s, 1),
                           "latency_ms_p50": round(float(np.percentile(np.array(lat_cap) * 1e3, 50)), 3),
                           "latency_ms_p99": round(float(np.percentile(np.array(lat_cap) * 1e3, 99)), 3)},
        "batch_autotuned": tuned,
        "cpu_baseline": cpu,
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
    cpu = None
    if not args.no_cpu_baseline:
        k = min(64, len(sources))
        cols = outk[:, :k].cpu().numpy().view(np.uint32)  # the many-source run's first k columns
        cpu = cpu_pool_baseline([("sssp", csr, int(x), 0) for x in sources[:k]],
                                f"SSSP from the first {k} of the {len(sources)} sources",
                                expect=lambda i: cols[:, i])
        if cpu["equal_device"] != f"{k}/{k}":
            raise SystemExit(f"many-source distances differ from the oracle: {cpu['equal_device']}")
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
        "cpu_baseline": cpu,
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


SERVE_RESIDENT = (  # name, scale, SSSP / PPR share among resident requests, lanes, rank lanes
    ("s18", 18, 0.50, 256, 256),
    ("s22", 22, 0.35, 256, 128),
    ("s24", 24, 0.15, 256, 64),
)
SERVE_TWIN_LANES = 64       # CC lanes of each symmetrised twin
SERVE_POOL = 64             # graphs of scale 10..14 uploaded on first use
SERVE_POOL_SHARE = 0.2      # share of requests on the uploaded pool
SERVE_LOADS = (0.5, 1.0, 2.0, 4.0)  # offered load, times the sequential capacity


def serve_requests(count, graphs, pool, seed):
    """Seeded request stream: 70% SSSP, 20% PPR (T = 20), 10% CC.  A request
    targets the uploaded pool with probability SERVE_POOL_SHARE (uniform
    graph), else a resident graph by its share; CC runs on the graph's
    symmetrised twin; sources are uniform among vertices with out-edges."""
    rng = np.random.default_rng(seed)
    names = [g[0] for g in SERVE_RESIDENT]
    share = np.array([g[2] for g in SERVE_RESIDENT])
    senders = {k: np.flatnonzero(c.outdeg > 0) for k, c in graphs.items()}
    reqs = []
    for _ in range(count):
        u = rng.random()
        prog = "cc" if u < 0.1 else ("sssp" if u < 0.8 else "ppr")
        if rng.random() < SERVE_POOL_SHARE:
            base = f"pool{int(rng.integers(0, len(pool)))}"
        else:
            base = names[int(rng.choice(len(names), p=share))]
        name = base + "u" if prog == "cc" else base
        src = 0 if prog == "cc" else int(rng.choice(senders[name]))
        reqs.append((name, prog, src))
    return reqs


def bench_serve(args, dev):
    """Request serving (continuous batching) against the plain path.

    Resident graphs: directed weighted R-MAT scales 18, 22 and 24 (edge
    factor 16), each with a symmetrised twin for CC; a seeded pool of scale
    10..14 graphs is uploaded on first use.  The plain path runs every request
    alone with vc_run, first come first served, on one stream; its measured
    capacity (requests/s) sets the offered loads.  For each load in
    SERVE_LOADS a fresh server (lane tables, rank-lane tables, worker
    threads; requests routed by expected completion) receives the same
    request stream with seeded Poisson arrivals; latency runs from arrival
    until the poller on the host sees the completion.  The plain path's
    latency at the same arrivals comes from a first-come-first-served queue
    over its measured service times."""
    import torch
    import rmatgen
    from paper_2010_01542_amd import Graph, Server, vc
    t = time.time()
    csrs = {}
    for name, scale, _, _, _ in SERVE_RESIDENT:
        csrs[name] = rmatgen.rmat(scale, 16, seed=rmatgen.BASE_SEED + scale, weighted=True, threads=args.gen_threads)
        csrs[name + "u"] = rmatgen.rmat(scale, 16, seed=rmatgen.BASE_SEED + scale, directed=False,
                                        threads=args.gen_threads)
    prng = np.random.default_rng(rmatgen.BASE_SEED + 8)
    pool = []
    for j in range(SERVE_POOL):
        sc, ef = int(prng.integers(10, 15)), int(prng.integers(8, 33))
        csrs[f"pool{j}"] = rmatgen.rmat(sc, ef, seed=rmatgen.BASE_SEED + 9000 + j, weighted=True)
        csrs[f"pool{j}u"] = rmatgen.rmat(sc, ef, seed=rmatgen.BASE_SEED + 9000 + j, directed=False)
        pool.append(f"pool{j}")
    log(f"generated serving graphs in {time.time() - t:.1f}s: " +
        ", ".join(f"{k} n={csrs[k].n} m={csrs[k].m}" for k in csrs if not k.startswith("pool")))
    resident = [k for k in csrs if not k.startswith("pool")]
    graphs = {k: Graph.from_csr(csrs[k], device=dev, symmetric=k.endswith("u")) for k in resident}
    lanes_of = {x[0]: x[3] for x in SERVE_RESIDENT}
    rank_lanes_of = {x[0]: x[4] for x in SERVE_RESIDENT}
    for x in SERVE_RESIDENT:
        lanes_of[x[0] + "u"] = SERVE_TWIN_LANES
        rank_lanes_of[x[0] + "u"] = 0
    reqs = serve_requests(args.requests, csrs, pool, rmatgen.BASE_SEED + 5)
    outs = []
    for name, prog, _ in reqs:
        outs.append(torch.empty(csrs[name].n, dtype=torch.float32 if prog == "ppr" else torch.int32, device=dev))

    def upload(name):
        return Graph.from_csr(csrs[name], device=dev, symmetric=name.endswith("u"))

    # plain path: every request alone, in order; pool graphs created on first use
    for name in resident:  # warm-up of every kind: transposes, workspaces
        for prog in ("sssp", "ppr") if not name.endswith("u") else ("cc",):
            graphs[name].run(prog, T=20)
    torch.cuda.synchronize()
    service = np.zeros(len(reqs))
    live = dict(graphs)
    t0 = time.perf_counter()
    for i, (name, prog, src) in enumerate(reqs):
        a = time.perf_counter()
        if name not in live:
            live[name] = upload(name)
        live[name].run(prog, outs[i], source=src, T=20)
        service[i] = time.perf_counter() - a
    base_s = time.perf_counter() - t0
    capacity = len(reqs) / base_s
    log(f"plain path: {len(reqs)} requests in {base_s:.2f}s ({capacity:.1f} requests/s)")

    def kind(i):
        name, prog, _ = reqs[i]
        return f"{prog}@{'pool' if name.startswith('pool') else name}"

    plain_by_kind = {}
    for i in range(len(reqs)):
        k = plain_by_kind.setdefault(kind(i), [0, 0.0])
        k[0] += 1
        k[1] += service[i] * 1e3
    plain_by_kind = {k: {"requests": v[0], "total_ms": round(v[1], 1), "mean_ms": round(v[1] / v[0], 3)}
                     for k, v in sorted(plain_by_kind.items())}
    log(f"plain path by kind: {json.dumps(plain_by_kind)}")
    checks = [i for i in range(len(reqs))][:: max(1, len(reqs) // 24)]
    ref = {i: outs[i].cpu() for i in checks}
    del live

    def run_server(arrivals):
        """Submits request i at arrivals[i] (seconds from the start) from this
        thread while a second thread polls completions (the poll call
        releases the interpreter lock), so latency is arrival to the moment
        the host sees the completion."""
        import threading
        srv = Server(workers=args.workers)
        ids = {k: srv.add_graph(g, lanes=lanes_of[k], rank_lanes=rank_lanes_of[k]) for k, g in graphs.items()}
        uploaded = {}
        lat = np.zeros(len(reqs))
        tick = {}
        state = {"got": 0, "lanes": 0, "error": None}
        lock = threading.Lock()
        t_start = time.perf_counter()

        def poller():
            while state["got"] < len(reqs) and state["error"] is None:
                for c in srv.poll(timeout_ms=50, cap=1024):
                    now = time.perf_counter() - t_start
                    with lock:
                        i = tick[c.ticket]
                    lat[i] = (now - arrivals[i]) * 1e3
                    state["lanes"] += c.lane >= 0
                    state["got"] += 1
                    if c.status != vc.OK:
                        state["error"] = c.message

        th = threading.Thread(target=poller)
        th.start()
        try:
            for i, (name, prog, src) in enumerate(reqs):
                wait = arrivals[i] - (time.perf_counter() - t_start)
                if wait > 0:
                    time.sleep(wait)
                if name not in ids:  # first use of a pool graph: upload and register
                    uploaded[name] = upload(name)
                    ids[name] = srv.add_graph(uploaded[name])
                with lock:
                    tick[srv.submit(ids[name], prog, outs[i], source=src, T=20)] = i
        finally:
            th.join()
        assert state["error"] is None, state["error"]
        span = time.perf_counter() - t_start
        info = srv.info()
        srv.close()
        for i in checks:
            assert torch.equal(outs[i].cpu(), ref[i]), f"served request {i} differs from its plain run"
        return span, lat, info, state["lanes"]

    def pct(a, q):
        return round(float(np.percentile(a, q)), 3)

    points = []
    for load in (args.loads or SERVE_LOADS):
        rate = load * capacity
        gaps = np.random.default_rng(rmatgen.BASE_SEED + 6).exponential(1.0 / rate, len(reqs))
        arrivals = np.cumsum(gaps) - gaps[0]
        span, lat, info, lanes_used = run_server(arrivals)
        fin, lat_plain = 0.0, np.zeros(len(reqs))
        for i in range(len(reqs)):
            fin = max(fin, arrivals[i]) + service[i]
            lat_plain[i] = (fin - arrivals[i]) * 1e3
        plain_span = fin
        by = {}
        for i in range(len(reqs)):
            by.setdefault(kind(i), []).append(lat[i])
        pt = {"offered_load": load, "arrival_rate_per_s": round(rate, 2),
              "requests_per_s": round(len(reqs) / span, 2),
              "latency_ms_p50": pct(lat, 50), "latency_ms_p99": pct(lat, 99),
              "plain_requests_per_s": round(len(reqs) / plain_span, 2),
              "plain_latency_ms_p50": pct(lat_plain, 50), "plain_latency_ms_p99": pct(lat_plain, 99),
              "lane_requests": lanes_used, "lane_supersteps": info["lane_supersteps"],
              "rank_supersteps": info["rank_supersteps"],
              "latency_ms_p50_by_kind": {k: pct(v, 50) for k, v in sorted(by.items())}}
        log(f"load {load}: {json.dumps(pt)}")
        points.append(pt)
    best = max(points, key=lambda x: x["requests_per_s"])
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on a seeded sample of the request stream; the plain
        # path's CC / SSSP results (kept in outs) must equal it
        pick = np.sort(np.random.default_rng(rmatgen.BASE_SEED + 10).choice(len(reqs), size=min(32, len(reqs)),
                                                                         replace=False))
        tasks = [(reqs[i][1], csrs[reqs[i][0]], reqs[i][2], 20) for i in pick]

        def expect(j):
            i = pick[j]
            return None if reqs[i][1] == "ppr" else outs[i].cpu().numpy().view(np.uint32)

        cpu = cpu_pool_baseline(tasks, f"a seeded sample of {len(tasks)} of the {len(reqs)} requests", expect)
        # throughput of the oracle serving the whole stream at that rate
        cpu["requests_per_s"] = cpu["queries_per_s"]
    return {
        "metric": "served requests/s (70% SSSP, 20% PPR T=20, 10% CC; resident R-MAT graphs and an uploaded pool)",
        "value": best["requests_per_s"], "unit": "requests/s", "n_gpus": 1, "steps": len(SERVE_LOADS), "warmup": 1,
        "ms_per_step": round(1e3 * len(reqs) / best["requests_per_s"], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32+f32", "data": "synthetic R-MAT (seeded)",
        "config": {"workload": f"serve-{len(reqs)}", "requests": len(reqs),
                   "graphs": {k: [csrs[k].n, csrs[k].m] for k in resident},
                   "uploaded_pool": {"graphs": SERVE_POOL, "scales": "10..14", "share": SERVE_POOL_SHARE},
                   "lanes": lanes_of, "rank_lanes": rank_lanes_of, "workers": args.workers,
                   "hw_queues": args.hw_queues},
        "plain": {"requests_per_s": round(capacity, 2), "by_kind": plain_by_kind},
        "speedup_vs_plain_at_best_load": round(best["requests_per_s"] / capacity, 2),
        "loads": points,
        "cpu_baseline": cpu,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="sssp-s26", choices=["sssp-s26", "cc-s22", "pr-s16", "batch", "multi", "serve", "combine"])
    ap.add_argument("--sources", type=int, default=256, help="multi workload: SSSP sources")
    ap.add_argument("--members", type=int, default=1024, help="batch workload: number of graphs")
    ap.add_argument("--requests", type=int, default=2000, help="serve workload: requests per offered load")
    ap.add_argument("--workers", type=int, default=4, help="serve workload: worker threads")
    ap.add_argument("--loads", type=float, nargs="*", default=None,
                    help="serve workload: offered loads (times the plain capacity); default 0.5 1 2 4")
    ap.add_argument("--hw-queues", type=int, default=None,
                    help="serve workload: hardware queues of the process (GPU_MAX_HW_QUEUES, at most 32); "
                         "lane tables, rank tables and workers each use their own stream")
    ap.add_argument("--scale", type=int, default=None, help="override the graph scale (same shape)")
    ap.add_argument("--schedule", default="auto", choices=["auto", "vertex", "edge", "pull", "blocked"])
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--f32-accumulate", action="store_true", help="binary32 PageRank combiner (float atomics)")
    ap.add_argument("--messages", default="f32", choices=["u64", "f32"],
                    help="PageRank message type with exact fixed-point sums: uint64 multiples of 2^-62, or "
                         "binary32 (VC_OPT_F32_MESSAGES); ignored with --f32-accumulate")
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
    from paper_2010_01542_amd import vc
    off_bytes = csr.off.dtype.itemsize
    n, m = csr.n, csr.m
    rank_options = vc.OPT_F32_ACCUMULATE if args.f32_accumulate else (
        vc.OPT_F32_MESSAGES if args.messages == "f32" else 0)
    kw = dict(schedule=args.schedule, tile=args.tile, options=0)
    # graph creation (upload, relabelled copy) and preparation (what a first
    # run builds: blocked layout, transpose, partitions), timed apart
    setup = {}
    t = time.perf_counter()
    off_t = torch.from_numpy(np.ascontiguousarray(csr.off)).to(dev)
    dst_t = torch.from_numpy(np.ascontiguousarray(csr.dst)).to(dev)
    w_t = None if csr.w is None else torch.from_numpy(np.ascontiguousarray(csr.w).view(np.int32)).to(dev)
    torch.cuda.synchronize()
    setup["upload_ms"] = round((time.perf_counter() - t) * 1e3, 1)
    t = time.perf_counter()
    g = Graph(off_t, dst_t, w_t, symmetric=args.workload == "cc-s22")
    setup["graph_create_ms"] = round((time.perf_counter() - t) * 1e3, 1)
    del off_t, dst_t, w_t
    log(f"uploaded in {setup['upload_ms']:.0f} ms, graph created in {setup['graph_create_ms']:.0f} ms")

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
        b.copy_(a)  # the copy whose counters scale FETCH_SIZE / WRITE_SIZE
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(5):
            b.copy_(a)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / 5
        log(f"calibration copy: 1 GiB read + 1 GiB written; five more take {ms:.3f} ms each = "
            f"{2 * 2**30 / (ms * 1e-3) / 1e12:.2f} TB/s")
        del a, b

    for prog, pk in jobs:
        t = time.perf_counter()
        pkw = dict(kw, options=rank_options) if prog in ("pagerank", "ppr") else dict(kw)
        if prog not in ("pagerank", "ppr") and pkw["schedule"] == "blocked":
            pkw["schedule"] = "auto"
        g.prepare(prog, **{k: v for k, v in pk.items() if k in ("T", "source")}, **pkw)
        setup[f"prepare_{prog}_ms"] = round((time.perf_counter() - t) * 1e3, 1)
    log(f"setup: {setup}")

    out_f = torch.empty(n, dtype=torch.float32, device=dev)
    out_u = torch.empty(n, dtype=torch.int32, device=dev)

    def step(timing):
        res = {}
        for prog, pk in jobs:
            out = out_f if prog in ("pagerank", "ppr") else out_u
            pkw = dict(kw)
            if prog in ("pagerank", "ppr"):
                pkw["options"] = rank_options
            elif kw["schedule"] == "blocked":
                pkw["schedule"] = "auto"  # the blocked form is PageRank's only
            _, st = g.run(prog, out, stats=True, timing=timing, **pk, **pkw)
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
        whole = np.concatenate([r["pagerank"].step_ms[:-1] for r in records])
        step_bytes = pr_superstep_bytes(n, m, off_bytes)
        step_ms = float(whole.mean())
        superstep = {"what": "broadcast+combine and the vertex update (rank write included)",
                     "algorithmic_bytes": int(step_bytes), "avg_ms": round(step_ms, 4),
                     "achieved": round(step_bytes / (step_ms * 1e-3) / 1e9, 1),
                     "frac": round(step_bytes / (step_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        sched = records[0]["pagerank"].schedule[0]
        kname = {1: "k_pr_scatter_vertex", 2: "k_pr_scatter_mp", 3: "k_pr_pull",
                 4: "k_pb_spread + k_pb_fold"}.get(int(sched), "?")
        if float(scat.max()) == 0.0:
            # a captured loop: its kernels cannot be timed apart, so the
            # roofline is the whole superstep's (graph time / T)
            roofline = {"bound": "hbm", "achieved": superstep["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": superstep["frac"], "traffic": None,
                        "kernel": f"captured superstep loop: {kname} + k_pr_apply per superstep",
                        "launches": int(whole.size), "avg_launch_ms": round(step_ms, 4),
                        "algorithmic_bytes_per_launch": int(step_bytes),
                        "gteps_per_launch": round(m / (step_ms * 1e-3) / 1e9, 2), "superstep": superstep}
        else:
            avg_ms = float(scat.mean())
            bytes_launch = pr_scatter_bytes(n, m, off_bytes)
            achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
            form = {3: "pull", 4: "blocked"}.get(int(sched))
            traffic = measured_traffic(csr.name, form, rank_options) if form else None
            roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                        "kernel": f"{kname} (PageRank broadcast+combine)", "launches": int(scat.size),
                        "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": int(bytes_launch),
                        "gteps_per_launch": round(m / (avg_ms * 1e-3) / 1e9, 2), "superstep": superstep}

    # hash-min CC: the vertex-centric and edge-centric work distributions
    # (and the dense forms) each run alone, every superstep in one form
    schedules = None
    if args.workload == "cc-s22":
        schedules = {}
        for sc in ("vertex", "edge", "pull", "blocked", "auto"):
            ms, sts = [], None
            for _ in range(3):
                _, sts = g.run("cc", out_u, schedule=sc, stats=True, timing=True)
                ms.append(sts.elapsed_ms)
            schedules[sc] = {"run_ms_median": round(float(np.median(ms)), 3),
                             "kernel_ms": round(float(sts.step_ms.sum()), 3),
                             "gteps": round(sts.edges_relaxed / (float(np.median(ms)) * 1e-3) / 1e9, 2),
                             "schedule_per_superstep": sts.schedule.tolist()}
        log(f"cc schedules: { {k: v['run_ms_median'] for k, v in schedules.items()} }")

    # the oracle: CPU baseline (one pinned host core) and the accuracy of this run
    cpu, accuracy, min_ref = None, {}, {}
    if not args.no_cpu_baseline:
        import oracle
        prev = os.sched_getaffinity(0)
        core = min(prev)
        os.sched_setaffinity(0, {core})  # one core, as the baseline states
        try:
            samples, msgs, secs = [], 0, 0.0
            for prog, pk in jobs:
                if prog in ("pagerank", "ppr"):
                    sample_T = 2  # the full T would take minutes of one core at scale 26
                    t = time.perf_counter()
                    ref = oracle.run_csr(prog, csr, T=sample_T, source=pk.get("source", 0))
                    dt = time.perf_counter() - t
                    msgs += sample_T * m
                    samples.append(f"{prog} {sample_T} supersteps ({sample_T * m} messages) {dt:.1f}s")
                    g.run(prog, out_f, T=sample_T, source=pk.get("source", 0), schedule=kw["schedule"],
                          tile=kw["tile"], options=rank_options)
                    diff = np.abs(out_f.cpu().numpy().astype(np.float64) - ref.values)
                    accuracy[prog] = {"T": sample_T, "l1": float(diff.sum()), "max_abs": float(diff.max()),
                                      "bars": {"l1": 1e-5, "max_abs": 1e-7},
                                      "note": "device run with the timed options, against the binary64 oracle"}
                else:
                    t = time.perf_counter()
                    ref = oracle.run_csr(prog, csr, source=pk.get("source", 0))
                    dt = time.perf_counter() - t
                    msgs += int(ref.messages.sum())
                    samples.append(f"{prog} to quiescence ({int(ref.messages.sum())} messages) {dt:.1f}s")
                    g.run(prog, out_u, source=pk.get("source", 0), schedule="auto", tile=kw["tile"])
                    exact = bool(np.array_equal(out_u.cpu().numpy().view(np.uint32), ref.values))
                    accuracy[prog] = {"bit_exact": exact,
                                      "frontier_equal": records[0][prog].frontier.tolist() == ref.senders.tolist()}
                    min_ref[prog] = ref
                secs += dt
        finally:
            os.sched_setaffinity(0, prev)
        cpu = {"value": round(msgs / secs / 1e9, 4), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": "oracle (single thread pinned to one core) over the full graph: " + "; ".join(samples)}
        log(f"cpu baseline: {cpu['value']} GTEPS in {secs:.1f}s; accuracy {accuracy}")

    # CC / SSSP: per-superstep algorithmic bytes against the HBM peak, with
    # |R_s| from the oracle's run
    for prog, ref in min_ref.items():
        st = records[0][prog]
        steps_ms = np.median(np.concatenate([r[prog].step_ms for r in records]).reshape(len(records), -1), axis=0)
        bs = min_superstep_bytes(n, off_bytes, prog == "sssp" and csr.w is not None, st.frontier.tolist(),
                                 st.edges.tolist(), ref.receivers.tolist(), dense0=prog == "cc")
        per = []
        for s, (b, ms) in enumerate(zip(bs, steps_ms.tolist())):
            if ms > 0:
                per.append({"s": s, "bytes": b, "ms": round(float(ms), 4),
                            "gbs": round(b / (ms * 1e-3) / 1e9, 1),
                            "frac": round(b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                            "schedule": int(st.schedule[s])})
        tot_b, tot_ms = sum(x["bytes"] for x in per), sum(x["ms"] for x in per)
        detail[prog]["hbm"] = {"per_superstep": per, "bytes": int(tot_b), "ms": round(tot_ms, 4),
                               "frac": round(tot_b / (tot_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4) if tot_ms else None}
        if dominant == prog and tot_ms:
            roofline = {"bound": "hbm", "achieved": round(tot_b / (tot_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": detail[prog]["hbm"]["frac"], "traffic": None,
                        "kernel": f"{prog} supersteps (broadcast+combine+update, every superstep of the run)",
                        "algorithmic_bytes_per_run": int(tot_b), "ms_per_run": round(tot_ms, 4)}

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
                   "schedule": args.schedule, "tile": args.tile or "default",
                   "rank_messages": "f32 (binary32, exact fixed-point sums)" if args.messages == "f32" and
                   not args.f32_accumulate else ("f32 atomics" if args.f32_accumulate else
                                                 "u64 (fixed point 2^-62, exact sums)")},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accuracy": accuracy,
        "pagerank_error": accuracy.get("pagerank"),
        "setup": setup,
        "schedules": schedules,
        "detail": detail,
        "host": host_info(),
        "device": torch.cuda.get_device_name(0),
        "python": platform.python_version(),
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
