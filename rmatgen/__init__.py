"""Seeded synthetic graph inputs, as CSR arrays.

This module produces inputs only; it is shared by the CPU oracle and the GPU
path and holds none of the vertex-centric method's arithmetic.

* ``rmat``: R-MAT graphs (a, b, c, d quadrant probabilities, no noise, no
  vertex relabelling) from a counter-based SplitMix64 stream, so a graph is a
  pure function of its seed.  Self-loops and duplicate edges are removed;
  undirected graphs are symmetrised.  Optional uint32 weights are uniform on
  [1, 255].
* ``from_edges``: the same clean-up applied to an explicit edge list.
* ``raw_csr``: a CSR that keeps every edge as given (duplicates, self-loops),
  for tests of multigraph semantics.
* Hand-shaped graphs (path, cycle, stars, cliques, complete digraph).
* ``workload``: the seeded benchmark graphs, by name.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_DIR, "rmat.cpp")
_LIB = os.path.join(_DIR, "librmat.so")
_lib = None

# Graph500 R-MAT quadrant probabilities (a, b, c); d = 1 - a - b - c.
GRAPH500_ABC = (0.57, 0.19, 0.19)
BASE_SEED = 20101542


def build() -> None:
    """Compiles the generator (host C++ with OpenMP)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    vp, i64, u64, dbl, cint = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
    lib.rmat_generate.restype = vp
    lib.rmat_generate.argtypes = [cint, dbl, dbl, dbl, dbl, u64, cint, cint, u64, cint]
    lib.rmat_from_edges.restype = vp
    lib.rmat_from_edges.argtypes = [i64, i64, vp, vp, cint, cint, u64]
    lib.rmat_num_vertices.restype = i64
    lib.rmat_num_vertices.argtypes = [vp]
    lib.rmat_num_edges.restype = i64
    lib.rmat_num_edges.argtypes = [vp]
    lib.rmat_has_weights.restype = cint
    lib.rmat_has_weights.argtypes = [vp]
    lib.rmat_copy_out.restype = cint
    lib.rmat_copy_out.argtypes = [vp, vp, vp, vp, vp]
    lib.rmat_free.restype = None
    lib.rmat_free.argtypes = [vp]
    lib.rmat_samples.restype = None
    lib.rmat_samples.argtypes = [cint, dbl, dbl, dbl, u64, u64, u64, vp, vp]
    _lib = lib
    return lib


@dataclass
class Csr:
    """A CSR graph in host memory (out-edges)."""

    n: int
    m: int
    off: np.ndarray  # int64 or int32, n + 1 entries
    dst: np.ndarray  # int32, m entries
    w: Optional[np.ndarray] = None  # uint32, m entries, or None
    name: str = ""

    @property
    def outdeg(self) -> np.ndarray:
        return np.diff(self.off.astype(np.int64))

    def off64(self) -> np.ndarray:
        return self.off.astype(np.int64, copy=False)

    def with_offsets(self, dtype) -> "Csr":
        if self.off.dtype == dtype:
            return self
        if dtype == np.int32 and self.m >= 2**31:
            raise ValueError("int32 offsets need fewer than 2^31 edges")
        return Csr(self.n, self.m, self.off.astype(dtype), self.dst, self.w, self.name)


def _take(handle, offset_dtype) -> Csr:
    lib = _load()
    try:
        n = lib.rmat_num_vertices(handle)
        m = lib.rmat_num_edges(handle)
        dst = np.empty(m, dtype=np.int32)
        w = np.empty(m, dtype=np.uint32) if lib.rmat_has_weights(handle) else None
        if offset_dtype == np.int32:
            off = np.empty(n + 1, dtype=np.int32)
            rc = lib.rmat_copy_out(handle, None, off.ctypes.data, dst.ctypes.data, None if w is None else w.ctypes.data)
        else:
            off = np.empty(n + 1, dtype=np.int64)
            rc = lib.rmat_copy_out(handle, off.ctypes.data, None, dst.ctypes.data, None if w is None else w.ctypes.data)
        if rc != 0:
            raise ValueError(f"rmat_copy_out failed ({rc})")
        return Csr(n, m, off, dst, w)
    finally:
        lib.rmat_free(handle)


def rmat(scale: int, edge_factor: float, a: float = GRAPH500_ABC[0], b: float = GRAPH500_ABC[1],
         c: float = GRAPH500_ABC[2], seed: int = BASE_SEED, directed: bool = True, weighted: bool = False,
         weight_seed: Optional[int] = None, offset_dtype=np.int64, threads: int = 0) -> Csr:
    """R-MAT graph with 2^scale vertices from edge_factor * 2^scale samples."""
    lib = _load()
    wseed = (seed + 1000) if weight_seed is None else weight_seed
    h = lib.rmat_generate(int(scale), float(edge_factor), float(a), float(b), float(c), int(seed) & (2**64 - 1),
                          int(directed), int(weighted), int(wseed) & (2**64 - 1), int(threads))
    if not h:
        raise ValueError("rmat_generate failed (bad arguments or out of memory)")
    g = _take(h, offset_dtype)
    g.name = f"rmat-s{scale}-ef{edge_factor:g}-{'dir' if directed else 'sym'}-seed{seed}"
    return g


def rmat_samples(scale: int, first: int, count: int, a=GRAPH500_ABC[0], b=GRAPH500_ABC[1], c=GRAPH500_ABC[2],
                 seed: int = BASE_SEED):
    """The raw (src, dst) R-MAT samples [first, first + count), before clean-up."""
    lib = _load()
    s = np.empty(count, dtype=np.uint32)
    d = np.empty(count, dtype=np.uint32)
    lib.rmat_samples(int(scale), float(a), float(b), float(c), int(seed) & (2**64 - 1), int(first), int(count),
                     s.ctypes.data, d.ctypes.data)
    return s, d


def from_edges(n: int, src, dst, directed: bool = True, weighted: bool = False, weight_seed: int = 7,
               offset_dtype=np.int64) -> Csr:
    """CSR from an edge list, with self-loops and duplicates removed."""
    lib = _load()
    s = np.ascontiguousarray(np.asarray(src, dtype=np.int64))
    d = np.ascontiguousarray(np.asarray(dst, dtype=np.int64))
    if s.shape != d.shape:
        raise ValueError("src and dst differ in length")
    h = lib.rmat_from_edges(int(n), int(s.size), s.ctypes.data, d.ctypes.data, int(directed), int(weighted),
                            int(weight_seed))
    if not h:
        raise ValueError("rmat_from_edges failed (vertex id out of range?)")
    return _take(h, offset_dtype)


def raw_csr(n: int, src, dst, w=None, offset_dtype=np.int64) -> Csr:
    """CSR that keeps every edge as given, grouped by source in input order."""
    s = np.asarray(src, dtype=np.int64)
    d = np.asarray(dst, dtype=np.int64)
    if s.size and (s.min() < 0 or s.max() >= n or d.min() < 0 or d.max() >= n):
        raise ValueError("vertex id out of range")
    order = np.argsort(s, kind="stable")
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(s, minlength=n), out=off[1:])
    ww = None if w is None else np.asarray(w, dtype=np.uint32)[order].copy()
    return Csr(n, int(s.size), off.astype(offset_dtype), d[order].astype(np.int32), ww)


# ----------------------------------------------------------------------------- hand-shaped graphs

def path(n: int, directed: bool = False, **kw) -> Csr:
    i = np.arange(n - 1)
    return from_edges(n, i, i + 1, directed=directed, **kw)


def cycle(n: int, **kw) -> Csr:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, directed=True, **kw)


def complete_digraph(n: int, **kw) -> Csr:
    s, d = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return from_edges(n, s.ravel(), d.ravel(), directed=True, **kw)


def out_star(leaves: int, **kw) -> Csr:
    """Vertex 0 points at vertices 1..leaves."""
    return from_edges(leaves + 1, np.zeros(leaves, dtype=np.int64), np.arange(1, leaves + 1), directed=True, **kw)


def in_star(leaves: int, **kw) -> Csr:
    """Vertices 1..leaves point at vertex 0."""
    return from_edges(leaves + 1, np.arange(1, leaves + 1), np.zeros(leaves, dtype=np.int64), directed=True, **kw)


def bi_star(leaves: int, **kw) -> Csr:
    """Hub 0 and leaves 1..leaves joined in both directions."""
    return from_edges(leaves + 1, np.zeros(leaves, dtype=np.int64), np.arange(1, leaves + 1), directed=False, **kw)


def cliques(sizes, isolated: int = 0, **kw) -> Csr:
    """Disjoint undirected cliques of the given sizes, then isolated vertices."""
    src, dst, base = [], [], 0
    for k in sizes:
        a, b = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
        src.append(base + a.ravel())
        dst.append(base + b.ravel())
        base += k
    n = base + isolated
    s = np.concatenate(src) if src else np.zeros(0, np.int64)
    d = np.concatenate(dst) if dst else np.zeros(0, np.int64)
    return from_edges(n, s, d, directed=False, **kw)


# ----------------------------------------------------------------------------- benchmark workloads

@dataclass(frozen=True)
class GraphSpec:
    scale: int
    edge_factor: float
    directed: bool
    weighted: bool
    offset_dtype: type
    seed: int


# PageRank graph: directed R-MAT scale 16, edge factor 16, int32 CSR.
# Hash-min CC graph: undirected (symmetrised) R-MAT scale 22, edge factor 16, int32 CSR.
# SSSP + PageRank graph: directed R-MAT scale 26, edge factor 16, int64 offsets, uint32 weights in [1, 255].
WORKLOADS = {
    "pr-s16": GraphSpec(16, 16, True, False, np.int32, BASE_SEED + 0),
    "cc-s22": GraphSpec(22, 16, False, False, np.int32, BASE_SEED + 1),
    "sssp-s26": GraphSpec(26, 16, True, True, np.int64, BASE_SEED + 2),
}


def workload(name: str, scale: Optional[int] = None, threads: int = 0) -> Csr:
    """The seeded benchmark graph `name`; `scale` overrides its size (same shape)."""
    spec = WORKLOADS[name]
    sc = spec.scale if scale is None else scale
    g = rmat(sc, spec.edge_factor, seed=spec.seed, directed=spec.directed, weighted=spec.weighted,
             offset_dtype=spec.offset_dtype, threads=threads)
    g.name = f"{name}@s{sc}"
    return g
