"""Many-source SSSP in one run (GPU): every column equals the oracle's SSSP
from that source, bit for bit."""
import numpy as np
import pytest

import oracle
import rmatgen

pytestmark = pytest.mark.gpu


def make(csr, **kw):
    from paper_2010_01542_amd import Graph
    return Graph.from_csr(csr, **kw)


def check_columns(csr, g, sources, **kw):
    out, st = g.run_multi_source(sources, stats=True, **kw)
    got = out.cpu().numpy().view(np.uint32)
    assert got.shape == (csr.n, len(sources))
    for i, s in enumerate(sources):
        ref = oracle.run("sssp", csr.n, csr.off, csr.dst, csr.w, source=int(s)).values
        assert np.array_equal(got[:, i], ref), (i, int(s))
    return got, st


@pytest.mark.parametrize("k", [1, 5, 64, 65, 200, 256])
@pytest.mark.parametrize("relabel", [True, False])
def test_multi_source_rmat(device, k, relabel):
    print(f"case multi-source rmat s11 k={k} relabel={relabel}", flush=True)
    d = rmatgen.rmat(11, 12, seed=k, weighted=True)
    rng = np.random.default_rng(k)
    sources = rng.integers(0, d.n, k)
    if k > 3:
        sources[1] = sources[0]  # a repeated source
        sources[2] = d.n - 1      # likely an isolated vertex
    check_columns(d, make(d, relabel=relabel), sources)


def test_multi_source_unit_weights_and_hand_graphs(device):
    d = rmatgen.rmat(10, 8, seed=3)
    check_columns(d, make(d), np.arange(0, 40))
    for c in (rmatgen.path(30, directed=True), rmatgen.out_star(300), rmatgen.cycle(17),
              rmatgen.raw_csr(6, [0, 0, 1, 2, 5], [1, 1, 2, 0, 5], [3, 1, 2, 9, 4])):
        check_columns(c, make(c), np.arange(c.n)[:64])


def test_multi_source_mid_size(device):
    d = rmatgen.rmat(15, 16, seed=44, weighted=True)
    sources = np.random.default_rng(1).integers(0, d.n, 256)
    got, st = check_columns(d, make(d), sources[:48])
    # the same sources in one 256-wide run agree with the narrower run
    out, _ = make(d).run_multi_source(sources)
    assert np.array_equal(out.cpu().numpy().view(np.uint32)[:, :48], got)


def test_multi_source_rejects_bad_arguments(device):
    from paper_2010_01542_amd import VcError
    g = make(rmatgen.path(4, directed=True))
    with pytest.raises(VcError):
        g.run_multi_source([4])
    with pytest.raises(VcError):
        g.run_multi_source(np.zeros(257, np.uint32))


@pytest.mark.parametrize("wmax", [20000, 40000, 65535, 1000000])
def test_multi_source_large_weights(device, wmax):
    """Weights up to wmax (the largest exactly wmax): distances well above
    2^16 come out exact in every column."""
    print(f"case multi-source large weights wmax={wmax}", flush=True)
    d = rmatgen.rmat(11, 12, seed=9, weighted=True)
    w = (d.w.astype(np.uint64) * 2654435761 % wmax + 1).astype(np.uint32)
    w[np.argmax(d.outdeg > 0)] = wmax
    c = rmatgen.Csr(d.n, d.m, d.off, d.dst, w)
    sources = np.random.default_rng(wmax).integers(0, c.n, 100)
    got, st = check_columns(c, make(c), sources)
    assert st.supersteps > 4
    if wmax >= 40000:
        assert got[got != 0xFFFFFFFF].max() > 0xFFFF
