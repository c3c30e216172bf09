"""Generic combiner (GPU): one superstep of message passing with combiners
that have no native atomic, against the oracle's flag-based mailboxes.

Bars: bit-exact mailboxes and flags for the integer, maximum and
(value, id) combiners, which are associative and commutative on their
inputs; for the binary64 sum, whose rounding depends on the order of
additions, |device - oracle| <= 2 k eps sum|m| per receiver of k messages
(the classical bound for two orders of the same sum), with exact flags.
Contention: every leaf of a 20,000-leaf in-star sends to the centre.  Both
forms run: pull when the senders' out-edges reach a tenth of the edges
(receivers fold their in-edges), push for sparser sender sets.
"""
import numpy as np
import pytest

import oracle
import rmatgen

pytestmark = pytest.mark.gpu

OPS = ["sum_u64", "prod_u64", "max_f64", "minarg", "sum_f64"]


def make(csr, **kw):
    from paper_2010_01542_amd import Graph
    return Graph.from_csr(csr, **kw)


def messages(op, n, rng):
    if op in ("sum_u64", "prod_u64"):
        return rng.integers(0, 2**64, n, dtype=np.uint64) | np.uint64(1)
    if op == "minarg":
        vals = rng.integers(-3, 4, n).astype(np.float32)  # many ties, decided by the id
        ids = rng.permutation(n).astype(np.uint32)
        return (ids.astype(np.uint64) << np.uint64(32)) | vals.view(np.uint32).astype(np.uint64)
    return rng.standard_normal(n).view(np.uint64)


def check(csr, g, op, rng, active=None):
    import torch
    words = messages(op, csr.n, rng)
    msg = torch.from_numpy(words.view(np.int64)).cuda()
    act = None if active is None else torch.from_numpy(active.astype(np.uint8)).cuda()
    box, has = g.combine(op, msg, act)
    box = box.cpu().numpy().view(np.uint64)
    has = has.cpu().numpy()
    ref, ref_has = oracle.combine(op, csr.n, csr.off, csr.dst, words, active)
    assert np.array_equal(has.astype(bool), ref_has), op
    assert np.all(box[~ref_has] == 0)
    if op != "sum_f64":
        assert np.array_equal(box[ref_has], ref[ref_has]), (op, int((box != ref).sum()))
        return
    src = np.repeat(np.arange(csr.n), np.diff(csr.off))
    keep = np.ones(src.size, bool) if active is None else active[src]
    dst = np.asarray(csr.dst)[keep]
    k = np.bincount(dst, minlength=csr.n)
    mag = np.zeros(csr.n)
    np.add.at(mag, dst, np.abs(words.view(np.float64)[src[keep]]))
    err = np.abs(box.view(np.float64) - ref.view(np.float64))
    assert np.all(err <= 2 * k * np.finfo(np.float64).eps * mag), float(err.max())


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("relabel", [True, False])
def test_combine_rmat(device, op, relabel):
    print(f"case combine rmat s11 op={op} relabel={relabel}", flush=True)
    d = rmatgen.rmat(11, 10, seed=31)
    g = make(d, relabel=relabel)
    rng = np.random.default_rng(7)
    check(d, g, op, rng)                                  # pull form (every vertex sends)
    check(d, g, op, rng, active=rng.random(d.n) < 0.3)    # pull form
    check(d, g, op, rng, active=rng.random(d.n) < 0.01)   # push form: few senders


@pytest.mark.parametrize("op", OPS)
def test_combine_contention_and_hand_graphs(device, op):
    print(f"case combine contention op={op}", flush=True)
    rng = np.random.default_rng(3)
    for c in (rmatgen.in_star(20000), rmatgen.out_star(3000), rmatgen.complete_digraph(40),
              rmatgen.raw_csr(5, [0, 0, 1, 1, 3, 3, 4], [1, 1, 1, 2, 3, 1, 4]), rmatgen.raw_csr(7, [], [])):
        g = make(c)
        check(c, g, op, rng)
        check(c, g, op, rng, active=rng.random(c.n) < 0.5)
        check(c, g, op, rng, active=rng.random(c.n) < 0.03)  # push form, still contended at the star centre


def test_combine_mid_size_exact(device):
    print("case combine rmat s16", flush=True)
    d = rmatgen.rmat(16, 16, seed=5)
    g = make(d)
    rng = np.random.default_rng(1)
    for op in ("sum_u64", "minarg"):
        check(d, g, op, rng)


def test_combine_rejects_bad_arguments(device):
    import torch
    from paper_2010_01542_amd import VcError
    g = make(rmatgen.path(4, directed=True))
    msg = torch.zeros(4, dtype=torch.int64, device="cuda")
    with pytest.raises(VcError):
        g.combine(9, msg)
    with pytest.raises(TypeError):
        g.combine("sum_u64", torch.zeros(3, dtype=torch.int64, device="cuda"))


def test_golden_neutral_combination(device):
    """Section III's case, written out by hand (tests/golden): messages whose
    combination equals the combiner's neutral value still leave the receiver
    flagged with that value; a receiver whose only sender is inactive, and
    vertices without in-edges, have no message."""
    import json
    import os
    import torch
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "neutral_combination.json")) as f:
        fx = json.load(f)
    gr = fx["graph"]
    csr = rmatgen.raw_csr(gr["n"], np.repeat(np.arange(gr["n"]), np.diff(gr["off"])), gr["dst"])
    g = make(csr)
    act = torch.from_numpy(np.array(gr["active"], np.uint8)).cuda()
    for case in fx["cases"]:
        print(f"case golden neutral combination {case['op']}", flush=True)
        words = np.array([int(x, 16) for x in case["msg"]], np.uint64)
        box, has = g.combine(case["op"], torch.from_numpy(words.view(np.int64)).cuda(), act)
        box = box.cpu().numpy().view(np.uint64)
        has = has.cpu().numpy().astype(bool)
        assert has.tolist() == [bool(h) for h in case["has"]], case["op"]
        for v, want in enumerate(case["box"]):
            assert int(box[v]) == (0 if want is None else int(want, 16)), (case["op"], v)
