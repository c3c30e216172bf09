"""Helpers shared by the GPU parity tests: run the HIP path, run the oracle,
compare them to the stated bars.

Bars:
* CC labels and SSSP distances: bit-exact, and the per-superstep frontier
  sizes |F_s| and message counts E_s, which the device counts in its
  compaction kernel, equal the oracle's (the superstep model is synchronous,
  so they are deterministic; the oracle's counts are pinned against dense
  min-plus relaxation in test_oracle_pins).
* PageRank / PPR: binary32 device ranks against the binary64 oracle,
  L1 = sum_v |r_dev - r_ora| <= 1e-5 and max_v |r_dev - r_ora| <= 1e-7.
  The device reports |F_s| = N and E_s = M for every PageRank superstep by
  definition (every vertex broadcasts), from the host, so those are not
  compared: such a comparison could not fail.
"""
import numpy as np

import oracle

L1_TOL = 1e-5
MAX_ABS_TOL = 1e-7


def run_gpu(graph, program, **kw):
    out, st = graph.run(program, stats=True, **kw)
    vals = out.cpu().numpy()
    if vals.dtype == np.int32:
        vals = vals.view(np.uint32)
    return vals, st


def rank_errors(dev, ref):
    diff = np.abs(dev.astype(np.float64) - ref)
    return float(diff.sum()), float(diff.max()) if diff.size else 0.0


def check_min(csr, graph, program, source=0, **kw):
    ref = oracle.run(program, csr.n, csr.off, csr.dst, csr.w if program == "sssp" else None, source=source)
    got, st = run_gpu(graph, program, source=source, **kw)
    assert np.array_equal(got, ref.values), f"{program}: {int((got != ref.values).sum())} values differ"
    assert st.supersteps == ref.supersteps, (st.supersteps, ref.supersteps)
    assert st.frontier.tolist() == ref.senders.tolist()
    assert st.edges.tolist() == ref.messages.tolist()
    return got, st, ref


def check_rank(csr, graph, program="pagerank", T=10, source=0, **kw):
    ref = oracle.run(program, csr.n, csr.off, csr.dst, T=T, source=source)
    got, st = run_gpu(graph, program, T=T, source=source, **kw)
    l1, mx = rank_errors(got, ref.values)
    print(f"{program} n={csr.n} m={csr.m} T={T} L1={l1:.3e} max_abs={mx:.3e}", flush=True)
    assert l1 <= L1_TOL and mx <= MAX_ABS_TOL, (l1, mx)
    assert st.supersteps == ref.supersteps
    return got, st, (l1, mx)
