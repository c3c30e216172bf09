"""The oracle pins must catch plausible mistakes.

Each case copies the oracle's C source, plants one mistake (a dropped term, a
wrong sign or comparison, an off-by-one, a wrong combiner), builds it into a
temporary library and checks that a small battery of independent pins --
closed forms, exact rationals, Dijkstra, union-find -- rejects it.  All of it
runs on the CPU.
"""
import json
import os
import subprocess

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components, dijkstra

import oracle
import rmatgen
from test_oracle_pins import hop_bounded_min

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "drop-damping": ("g->rank[v] = teleport + g->d * sum;", "g->rank[v] = teleport + sum;"),
    "teleport-not-divided": ("(1.0 - g->d) / (double)g->n;", "(1.0 - g->d);"),
    "wrong-outdegree": ("g->rank[v] / (double)deg", "g->rank[v] / (double)(deg + 1)"),
    "sum-overwrites": ("g->fmsg_next[u] = g->fmsg_next[u] + m;", "g->fmsg_next[u] = m;"),
    "min-becomes-max": ("if (m < g->umsg_next[u]) g->umsg_next[u] = m;",
                        "if (m > g->umsg_next[u]) g->umsg_next[u] = m;"),
    "weight-ignored": ("deliver_min(g, g->dst[e], base + we);", "deliver_min(g, g->dst[e], base + 1u);"),
    "no-reactivation": ("if (g.halted[v] && !g.has_cur[v]) continue;", "if (g.halted[v]) continue;"),
    "one-update-too-many": ("if (s < g->T) {", "if (s <= g->T) {"),
    "cc-accepts-equal": ("g->has_cur[v] && g->umsg_cur[v] < g->label[v]) {\n    g->label[v] = g->umsg_cur[v];\n    broadcast_min",
                         "g->has_cur[v] && g->umsg_cur[v] <= g->label[v] + 1) {\n    g->label[v] = g->umsg_cur[v];\n    broadcast_min"),
    "stale-mailbox": ("    memset(g.has_next, 0, nn);\n", ""),
    "first-message-combined-with-zero": ("mailbox[u] = msg[v]; /* first message: stored, flag set */",
                                         "mailbox[u] = combine_words(op, 0, msg[v]);"),
    "minarg-tie-to-larger-id": ("(b == a && ib < ia)", "(b == a && ib > ia)"),
    "max-becomes-min": ("word_f64(msg) > word_f64(stored)", "word_f64(msg) < word_f64(stored)"),
    "inactive-vertices-send": ("if (active && !active[v]) continue;", "if (active && !active[v] && v < 0) continue;"),
    # per-superstep counts: a message not counted, receivers read from the wrong mailbox flags
    "messages-miscounted": ("    deliver_min(g, g->dst[e], m);\n    g->messages++;",
                            "    deliver_min(g, g->dst[e], m);\n    if (e > g->off[v]) g->messages++;"),
    "receivers-from-current-flags": ("receivers += g.has_next[v];", "receivers += g.has_cur[v];"),
    # Section III's failure: "received" read as "mailbox differs from the neutral value"
    "received-means-not-neutral": ("  }\n  return ORACLE_OK;\n}\n\n/* Library version tag",
                                   "  }\n  for (int64_t u = 0; u < n; ++u) has[u] = has[u] && mailbox[u] != 0;\n"
                                   "  return ORACLE_OK;\n}\n\n/* Library version tag"),
}


def _pins_pass(lib) -> bool:
    """True when the library passes every pin of the battery."""
    d = 0.85
    try:
        # PageRank closed forms: in-star and bidirectional star
        L = 5
        n = L + 1
        base = (1 - d) / n
        r = oracle.run_csr("pagerank", rmatgen.in_star(L), T=3, lib=lib).values
        if not (np.allclose(r[1:], base, rtol=1e-13) and abs(r[0] - (base + d * L * base)) < 1e-13):
            return False
        h, lo = 1.0 / n, 1.0 / n
        for _ in range(4):
            h, lo = base + d * L * lo, base + d * h / L
        r = oracle.run_csr("pagerank", rmatgen.bi_star(L), T=4, lib=lib).values
        if not (abs(r[0] - h) < 1e-13 and np.allclose(r[1:], lo, rtol=1e-13)):
            return False
        # PageRank on a multigraph vs dense iteration (with a dangling vertex)
        g = rmatgen.raw_csr(5, [0, 0, 0, 1, 1, 2, 3], [1, 1, 0, 2, 2, 3, 0])
        deg = np.diff(g.off)
        p = np.zeros((5, 5))
        np.add.at(p, (np.repeat(np.arange(5), deg), g.dst), 1.0 / np.repeat(deg, deg))
        x = np.full(5, 0.2)
        for _ in range(6):
            x = (1 - d) / 5 + d * p.T @ x
        r = oracle.run("pagerank", 5, g.off, g.dst, T=6, lib=lib)
        if r.supersteps != 7 or np.max(np.abs(r.values - x)) > 1e-14:
            return False
        # CC vs connected components on a seeded random graph
        rng = np.random.default_rng(1)
        s, t = rng.integers(0, 300, 250), rng.integers(0, 300, 250)
        g = rmatgen.from_edges(300, s, t, directed=False)
        _, lab = connected_components(csr_matrix((np.ones(250), (s, t)), shape=(300, 300)), directed=False)
        mins = np.full(lab.max() + 1, 300)
        np.minimum.at(mins, lab, np.arange(300))
        r = oracle.run_csr("cc", g, lib=lib)
        if not np.array_equal(r.values, mins[lab]):
            return False
        # its per-superstep senders, messages and receivers against dense label propagation
        arcs = [(u, v, 0) for u, v in zip(np.repeat(np.arange(g.n), g.outdeg).tolist(), g.dst.tolist())]
        if (r.senders.tolist(), r.messages.tolist(), r.receivers.tolist()) != hop_bounded_min(
                g.n, arcs, np.arange(g.n), np.ones(g.n, bool)):
            return False
        # SSSP vs Dijkstra on a seeded weighted R-MAT graph
        g = rmatgen.rmat(9, 8, seed=4, weighted=True)
        a = csr_matrix((g.w.astype(float), (np.repeat(np.arange(g.n), g.outdeg), g.dst)), shape=(g.n, g.n))
        ref = dijkstra(a, indices=0)
        got = oracle.run_csr("sssp", g, source=0, lib=lib).values
        fin = np.isfinite(ref)
        if not (np.array_equal(got[fin], ref[fin].astype(np.uint32)) and np.all(got[~fin] == oracle.UNREACHED)):
            return False
        # CC path closed form, including the superstep count
        r = oracle.run_csr("cc", rmatgen.path(6), lib=lib)
        if r.senders.tolist() != [6, 5, 4, 3, 2, 1, 0]:
            return False
        # combiners vs numpy ufunc.at and brute force (first message stored, no neutral value)
        g = rmatgen.rmat(8, 6, seed=11)
        rng = np.random.default_rng(11)
        act = rng.random(g.n) < 0.7
        src = np.repeat(np.arange(g.n), np.diff(g.off))
        keep = act[src]
        msg = rng.integers(0, 2**64, g.n, dtype=np.uint64) | np.uint64(1)
        box, has = oracle.combine("prod_u64", g.n, g.off, g.dst, msg, act, lib=lib)
        ref = np.ones(g.n, np.uint64)
        np.multiply.at(ref, g.dst[keep], msg[src[keep]])
        if not (np.array_equal(has, np.bincount(g.dst[keep], minlength=g.n) > 0) and np.array_equal(box[has], ref[has])):
            return False
        vals = rng.standard_normal(g.n)
        box, has = oracle.combine("max_f64", g.n, g.off, g.dst, vals, act, lib=lib)
        ref = np.full(g.n, -np.inf)
        np.maximum.at(ref, g.dst[keep], vals[src[keep]])
        if not np.array_equal(box.view(np.float64)[has], ref[has]):
            return False
        v32 = rng.integers(-2, 3, g.n).astype(np.float32)
        ids = rng.permutation(g.n).astype(np.uint32)
        words = (ids.astype(np.uint64) << np.uint64(32)) | v32.view(np.uint32).astype(np.uint64)
        box, has = oracle.combine("minarg", g.n, g.off, g.dst, words, act, lib=lib)
        for u in range(g.n):
            senders = src[(g.dst == u) & act[src]]
            if senders.size and box[u] != words[min(senders, key=lambda v: (v32[v], ids[v]))]:
                return False
        # Section III's neutral-value case, written out by hand (tests/golden)
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "neutral_combination.json")) as f:
            fx = json.load(f)
        gr = fx["graph"]
        for case in fx["cases"]:
            words = np.array([int(x, 16) for x in case["msg"]], np.uint64)
            box, has = oracle.combine(case["op"], gr["n"], gr["off"], gr["dst"], words, np.array(gr["active"], bool),
                                      lib=lib)
            if has.tolist() != [bool(h) for h in case["has"]]:
                return False
            if any(w is not None and int(box[v]) != int(w, 16) for v, w in enumerate(case["box"])):
                return False
    except oracle.OracleError:
        return False
    return True


def test_unmutated_oracle_passes_battery():
    assert _pins_pass(oracle._load())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of {name} not unique"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-w", "-fPIC", "-shared", "-o", str(so), str(path)])
    assert not _pins_pass(oracle.load_variant(str(so))), f"mutant {name} survived the pins"
