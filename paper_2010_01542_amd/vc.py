"""ctypes binding of libvc (include/vc.h): argument marshalling only.

Every step of a run executes in libvc's HIP kernels; PyTorch supplies device
memory and streams.  There is no CPU fallback: if the library cannot be
loaded, importing the binding's entry points raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libvc.so")

PAGERANK, CC_HASHMIN, SSSP, PPR = 0, 1, 2, 3
PROGRAMS = {"pagerank": PAGERANK, "pr": PAGERANK, "cc": CC_HASHMIN, "cc_hashmin": CC_HASHMIN, "sssp": SSSP,
            "ppr": PPR}
SCHED_AUTO, SCHED_VERTEX, SCHED_EDGE, SCHED_PULL, SCHED_BLOCKED = 0, 1, 2, 3, 4
SCHEDULES = {"auto": SCHED_AUTO, "vertex": SCHED_VERTEX, "edge": SCHED_EDGE, "pull": SCHED_PULL,
             "blocked": SCHED_BLOCKED}
IDX_I32, IDX_I64 = 0, 1
GRAPH_BORROW, GRAPH_VALIDATE, GRAPH_SYMMETRIC, GRAPH_NO_RELABEL = 1, 2, 4, 8
OPT_NO_HUB_AGGREGATION, OPT_NO_TEST_BEFORE_ATOMIC, OPT_F32_ACCUMULATE, OPT_GRAPH_CAPTURE = 1, 2, 4, 8
OPT_F32_MESSAGES = 16
UNREACHED = 0xFFFFFFFF
ROUTE_AUTO, ROUTE_LANES, ROUTE_WORKER = 0, 1, 2
COMBINERS = {"sum_u64": 0, "prod_u64": 1, "max_f64": 2, "minarg": 3, "sum_f64": 4}
ROUTES = {"auto": ROUTE_AUTO, "lanes": ROUTE_LANES, "worker": ROUTE_WORKER}

OK, ERR_INVALID_ARG, ERR_BAD_GRAPH, ERR_OUT_OF_MEMORY, ERR_HIP, ERR_UNSUPPORTED, ERR_NOT_CONVERGED = range(7)
ABI_VERSION = 1
EXPORTS = ("vc_graph_create", "vc_graph_destroy", "vc_graph_footprint", "vc_run", "vc_params_default",
           "vc_status_string", "vc_last_error", "vc_abi_version", "vc_batch_create", "vc_batch_layout",
           "vc_batch_run", "vc_batch_destroy", "vc_run_multi_source", "vc_graph_autotune", "vc_batch_autotune",
           "vc_server_create", "vc_server_add_graph", "vc_server_submit", "vc_server_poll", "vc_server_drain",
           "vc_server_info_get", "vc_server_destroy", "vc_combine", "vc_graph_prepare", "vc_run_noalloc")
NOALLOC_SCRATCH_BYTES = 64 << 20  # VC_NOALLOC_SCRATCH_BYTES


class GraphDesc(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("num_vertices", ctypes.c_int64),
                ("num_edges", ctypes.c_int64), ("offset_type", ctypes.c_int), ("offsets", ctypes.c_void_p),
                ("dst", ctypes.c_void_p), ("weights", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_supersteps", ctypes.c_int32), ("damping", ctypes.c_double),
                ("source", ctypes.c_uint32), ("schedule", ctypes.c_int), ("tile", ctypes.c_int32),
                ("options", ctypes.c_uint32), ("pull_fraction", ctypes.c_float)]


class StatsStruct(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("supersteps", ctypes.c_int32),
                ("edges_relaxed", ctypes.c_int64), ("elapsed_ms", ctypes.c_double), ("capacity", ctypes.c_int32),
                ("frontier", ctypes.c_void_p), ("edges", ctypes.c_void_p), ("scatter_ms", ctypes.c_void_p),
                ("step_ms", ctypes.c_void_p), ("schedule", ctypes.c_void_p)]


class BatchQuery(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("program", ctypes.c_int), ("source", ctypes.c_uint32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("workers", ctypes.c_int32), ("hbm_budget", ctypes.c_uint64)]


class Request(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("graph", ctypes.c_int32), ("program", ctypes.c_int),
                ("route", ctypes.c_int), ("params", Params), ("out", ctypes.c_void_p), ("tag", ctypes.c_uint64)]


class CompletionStruct(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int),
                ("supersteps", ctypes.c_int32), ("lane", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("queue_ms", ctypes.c_double), ("service_ms", ctypes.c_double), ("message", ctypes.c_char * 120)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("graphs", ctypes.c_int32), ("hbm_budget", ctypes.c_uint64),
                ("bytes_reserved", ctypes.c_uint64), ("bytes_held", ctypes.c_uint64), ("submitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("lane_supersteps", ctypes.c_int64),
                ("lane_push_supersteps", ctypes.c_int64), ("lane_requests", ctypes.c_int64),
                ("rank_supersteps", ctypes.c_int64), ("rank_requests", ctypes.c_int64)]


class VcError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Loads libvc.so, building it first only when no build exists."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(path)
    vp, i32 = ctypes.c_void_p, ctypes.c_int
    lib.vc_graph_create.restype = i32
    lib.vc_graph_create.argtypes = [ctypes.POINTER(GraphDesc), vp, ctypes.POINTER(vp)]
    lib.vc_graph_destroy.restype = i32
    lib.vc_graph_destroy.argtypes = [vp]
    lib.vc_graph_footprint.restype = i32
    lib.vc_graph_footprint.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    lib.vc_run.restype = i32
    lib.vc_run.argtypes = [vp, i32, ctypes.POINTER(Params), vp, vp, ctypes.POINTER(StatsStruct)]
    lib.vc_run_noalloc.restype = i32
    lib.vc_run_noalloc.argtypes = [vp, i32, ctypes.POINTER(Params), vp, vp, ctypes.POINTER(StatsStruct)]
    lib.vc_graph_prepare.restype = i32
    lib.vc_graph_prepare.argtypes = [vp, i32, ctypes.POINTER(Params), vp]
    lib.vc_params_default.restype = None
    lib.vc_params_default.argtypes = [ctypes.POINTER(Params)]
    lib.vc_status_string.restype = ctypes.c_char_p
    lib.vc_status_string.argtypes = [i32]
    lib.vc_last_error.restype = ctypes.c_char_p
    lib.vc_last_error.argtypes = []
    lib.vc_abi_version.restype = i32
    lib.vc_batch_create.restype = i32
    lib.vc_batch_create.argtypes = [ctypes.POINTER(GraphDesc), ctypes.POINTER(BatchQuery), ctypes.c_int32,
                                    ctypes.c_uint32, vp, ctypes.POINTER(vp)]
    lib.vc_batch_layout.restype = i32
    lib.vc_batch_layout.argtypes = [vp, vp]
    lib.vc_batch_run.restype = i32
    lib.vc_batch_run.argtypes = [vp, ctypes.POINTER(Params), vp, vp, ctypes.POINTER(StatsStruct)]
    lib.vc_batch_destroy.restype = i32
    lib.vc_batch_destroy.argtypes = [vp]
    lib.vc_graph_autotune.restype = i32
    lib.vc_graph_autotune.argtypes = [vp, i32, ctypes.POINTER(Params), vp, ctypes.POINTER(Params)]
    lib.vc_batch_autotune.restype = i32
    lib.vc_batch_autotune.argtypes = [vp, ctypes.POINTER(Params), vp, ctypes.POINTER(Params)]
    lib.vc_run_multi_source.restype = i32
    lib.vc_run_multi_source.argtypes = [vp, vp, ctypes.c_int32, ctypes.POINTER(Params), vp, vp,
                                        ctypes.POINTER(StatsStruct)]
    lib.vc_combine.restype = i32
    lib.vc_combine.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    lib.vc_server_create.restype = i32
    lib.vc_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]
    lib.vc_server_add_graph.restype = i32
    lib.vc_server_add_graph.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
    lib.vc_server_submit.restype = i32
    lib.vc_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    lib.vc_server_poll.restype = i32
    lib.vc_server_poll.argtypes = [vp, ctypes.POINTER(CompletionStruct), ctypes.c_int32, ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32)]
    lib.vc_server_drain.restype = i32
    lib.vc_server_drain.argtypes = [vp]
    lib.vc_server_info_get.restype = i32
    lib.vc_server_info_get.argtypes = [vp, ctypes.POINTER(ServerInfo)]
    lib.vc_server_destroy.restype = i32
    lib.vc_server_destroy.argtypes = [vp]
    if lib.vc_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{path}: ABI version {lib.vc_abi_version()} != {ABI_VERSION}; rebuild the library")
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != OK:
        lib = load()
        raise VcError(status, where, lib.vc_last_error().decode() or lib.vc_status_string(status).decode())


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _program(p) -> int:
    return PROGRAMS[p.lower()] if isinstance(p, str) else int(p)


@dataclass
class Stats:
    supersteps: int
    edges_relaxed: int
    elapsed_ms: float
    frontier: np.ndarray
    edges: np.ndarray
    scatter_ms: Optional[np.ndarray] = None
    step_ms: Optional[np.ndarray] = None
    schedule: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)


class Graph:
    """A CSR graph resident on the current GPU (vc_graph_create).

    offsets: int32 / int64 tensor of N+1 entries, dst: int32 tensor of M
    entries, weights: optional int32 / uint32 tensor of M entries (read as
    uint32); all on the current CUDA (HIP) device and contiguous.  With
    borrow=True the tensors are kept referenced by this object and must not be
    modified while it lives.
    """

    def __init__(self, offsets, dst, weights=None, *, borrow: bool = True, validate: bool = False,
                 symmetric: bool = False, relabel: bool = True, stream=None):
        import torch
        lib = load()
        for name, t in (("offsets", offsets), ("dst", dst), ("weights", weights)):
            if t is None:
                continue
            if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
                raise TypeError(f"{name} must be a contiguous CUDA tensor")
        if offsets.dtype not in (torch.int32, torch.int64):
            raise TypeError("offsets must be int32 or int64")
        if dst.dtype != torch.int32:
            raise TypeError("dst must be int32")
        if weights is not None and weights.dtype not in (torch.int32, getattr(torch, "uint32", torch.int32)):
            raise TypeError("weights must be int32 or uint32")
        n = offsets.numel() - 1
        m = dst.numel()
        if weights is not None and weights.numel() != m:
            raise ValueError("weights and dst differ in length")
        desc = GraphDesc(ctypes.sizeof(GraphDesc),
                         (GRAPH_BORROW if borrow else 0) | (GRAPH_VALIDATE if validate else 0) |
                         (GRAPH_SYMMETRIC if symmetric else 0) | (0 if relabel else GRAPH_NO_RELABEL),
                         n, m, IDX_I64 if offsets.dtype == torch.int64 else IDX_I32, offsets.data_ptr(),
                         dst.data_ptr() if m else None, weights.data_ptr() if weights is not None and m else None)
        handle = ctypes.c_void_p()
        _check(lib.vc_graph_create(ctypes.byref(desc), _stream_handle(stream), ctypes.byref(handle)),
               "vc_graph_create")
        self._h = handle
        self._keep = (offsets, dst, weights) if borrow and not relabel else None
        self.n, self.m = n, m
        self.weighted = weights is not None
        self.device = offsets.device

    @classmethod
    def from_csr(cls, csr, device=None, **kw) -> "Graph":
        """Uploads an rmatgen.Csr (host arrays) and creates the graph (borrowed)."""
        import torch
        device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        off = torch.from_numpy(np.ascontiguousarray(csr.off)).to(device)
        dst = torch.from_numpy(np.ascontiguousarray(csr.dst)).to(device)
        w = None
        if csr.w is not None:
            w = torch.from_numpy(np.ascontiguousarray(csr.w).view(np.int32)).to(device)
        torch.cuda.synchronize(device)
        return cls(off, dst, w, borrow=True, **kw)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().vc_graph_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._keep = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def footprint(self, program="sssp"):
        held, run = ctypes.c_size_t(), ctypes.c_size_t()
        _check(load().vc_graph_footprint(self._h, _program(program), ctypes.byref(held), ctypes.byref(run)),
               "vc_graph_footprint")
        return held.value, run.value

    def prepare(self, program, *, T: int = 10, source: int = 0, schedule="auto", tile: int = 0, options: int = 0,
                stream=None):
        """vc_graph_prepare: builds what a first run with these parameters would build."""
        prog = _program(program)
        p = _params(T if prog in (PAGERANK, PPR) else 0, 0.85, source, schedule, tile, options)
        _check(load().vc_graph_prepare(self._h, prog, ctypes.byref(p), _stream_handle(stream)), "vc_graph_prepare")

    def autotune(self, program, *, T: int = 10, damping: float = 0.85, source: int = 0, stream=None) -> dict:
        """vc_graph_autotune: picks and keeps the fastest distribution for `program`."""
        prog = _program(program)
        base = _params(T if prog in (PAGERANK, PPR) else 0, damping, source, "auto", 0, 0)
        best = Params()
        _check(load().vc_graph_autotune(self._h, prog, ctypes.byref(base), _stream_handle(stream), ctypes.byref(best)),
               "vc_graph_autotune")
        return _params_dict(best)

    def run_multi_source(self, sources, out=None, *, max_supersteps: int = 0, tile: int = 0, stream=None,
                         stats: bool = False, timing: bool = False, capacity: int = 4096):
        """vc_run_multi_source: distances from every source, as an (N, k) int32-stored uint32 tensor."""
        import torch
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.uint32))
        k = int(src.size)
        if out is None:
            out = torch.empty((self.n, k), dtype=torch.int32, device=self.device)
        if not out.is_cuda or not out.is_contiguous() or out.numel() != self.n * k or out.element_size() != 4:
            raise TypeError("out must be a contiguous CUDA tensor of N * k 4-byte elements")
        p = _params(max_supersteps, 0.85, 0, "pull", tile, 0)
        st, arrays = _stats_struct(stats or timing, timing, capacity)
        rc = load().vc_run_multi_source(self._h, src.ctypes.data, k, ctypes.byref(p), out.data_ptr(),
                                        _stream_handle(stream), ctypes.byref(st) if st is not None else None)
        _check(rc, "vc_run_multi_source")
        return out, _stats_result(st, arrays, capacity)

    def combine(self, op, msg, active=None, mailbox=None, has=None, stream=None):
        """vc_combine: one superstep with combiner `op` (COMBINERS); msg: N 8-byte
        words (int64 / uint64 / float64 tensor), active: optional N uint8 / bool.
        Returns (mailbox as int64 words, has as int32)."""
        import torch
        code = COMBINERS[op] if isinstance(op, str) else int(op)
        if not msg.is_cuda or not msg.is_contiguous() or msg.numel() != self.n or msg.element_size() != 8:
            raise TypeError("msg must be a contiguous CUDA tensor of N 8-byte elements")
        if active is not None:
            if active.dtype == torch.bool:
                active = active.to(torch.uint8)
            if not active.is_cuda or not active.is_contiguous() or active.numel() != self.n or active.element_size() != 1:
                raise TypeError("active must be a contiguous CUDA tensor of N bytes")
        if mailbox is None:
            mailbox = torch.empty(self.n, dtype=torch.int64, device=self.device)
        if has is None:
            has = torch.empty(self.n, dtype=torch.int32, device=self.device)
        _check(load().vc_combine(self._h, code, msg.data_ptr(), None if active is None else active.data_ptr(),
                                 mailbox.data_ptr(), has.data_ptr(), _stream_handle(stream)), "vc_combine")
        return mailbox, has

    def run(self, program, out=None, *, T: int = 10, damping: float = 0.85, source: int = 0,
            max_supersteps: int = 0, schedule="auto", tile: int = 0, options: int = 0, pull_fraction: float = 0.0,
            stream=None, stats: bool = False, timing: bool = False, capacity: int = 4096):
        """vc_run: returns (out, Stats | None).  out: float32 ranks or int32-stored uint32 labels."""
        import torch
        lib = load()
        prog = _program(program)
        rank = prog in (PAGERANK, PPR)
        if out is None:
            out = torch.empty(self.n, dtype=torch.float32 if rank else torch.int32, device=self.device)
        if not out.is_cuda or not out.is_contiguous() or out.numel() != self.n or out.element_size() != 4:
            raise TypeError("out must be a contiguous CUDA tensor of N 4-byte elements")
        p = _params(T if rank else max_supersteps, damping, source, schedule, tile, options, pull_fraction)
        st, arrays = _stats_struct(stats or timing, timing, capacity)
        rc = lib.vc_run(self._h, prog, ctypes.byref(p), out.data_ptr(), _stream_handle(stream),
                        ctypes.byref(st) if st is not None else None)
        _check(rc, "vc_run")
        return out, _stats_result(st, arrays, capacity)

    def run_noalloc(self, program, out, *, T: int = 10, damping: float = 0.85, source: int = 0,
                    max_supersteps: int = 0, schedule="auto", tile: int = 0, options: int = 0,
                    pull_fraction: float = 0.0, stream=None, stats: bool = False, capacity: int = 4096):
        """vc_run_noalloc: as run(), into a caller-supplied out tensor; the
        library allocates no device memory for it."""
        prog = _program(program)
        rank = prog in (PAGERANK, PPR)
        if out is None or not out.is_cuda or not out.is_contiguous() or out.numel() != self.n or \
                out.element_size() != 4:
            raise TypeError("out must be a contiguous CUDA tensor of N 4-byte elements")
        p = _params(T if rank else max_supersteps, damping, source, schedule, tile, options, pull_fraction)
        st, arrays = _stats_struct(stats, False, capacity)
        rc = load().vc_run_noalloc(self._h, prog, ctypes.byref(p), out.data_ptr(), _stream_handle(stream),
                                   ctypes.byref(st) if st is not None else None)
        _check(rc, "vc_run_noalloc")
        return out, _stats_result(st, arrays, capacity)


def _params(steps, damping, source, schedule, tile, options, pull_fraction=0.0) -> Params:
    p = Params()
    load().vc_params_default(ctypes.byref(p))
    p.max_supersteps = int(steps)
    p.damping = float(damping)
    p.source = int(source)
    p.schedule = SCHEDULES[schedule] if isinstance(schedule, str) else int(schedule)
    p.tile = int(tile)
    p.options = int(options)
    p.pull_fraction = float(pull_fraction)
    return p


def _params_dict(p: Params) -> dict:
    inv = {v: k for k, v in SCHEDULES.items()}
    return {"schedule": inv.get(p.schedule, p.schedule), "tile": p.tile, "pull_fraction": round(p.pull_fraction, 4),
            "capture": bool(p.options & OPT_GRAPH_CAPTURE)}


def _stats_struct(want: bool, timing: bool, capacity: int):
    if not want:
        return None, {}
    cap = int(capacity)
    arrays = {"frontier": np.zeros(cap, np.int64), "edges": np.zeros(cap, np.int64),
              "schedule": np.zeros(cap, np.int32)}
    if timing:
        arrays["scatter_ms"] = np.zeros(cap, np.float32)
        arrays["step_ms"] = np.zeros(cap, np.float32)
    st = StatsStruct(ctypes.sizeof(StatsStruct), 0, 0, 0.0, cap, arrays["frontier"].ctypes.data,
                     arrays["edges"].ctypes.data, arrays["scatter_ms"].ctypes.data if timing else None,
                     arrays["step_ms"].ctypes.data if timing else None, arrays["schedule"].ctypes.data)
    return st, arrays


def _stats_result(st, arrays, capacity):
    if st is None:
        return None
    k = min(st.supersteps, int(capacity))
    timing = "scatter_ms" in arrays
    return Stats(st.supersteps, st.edges_relaxed, st.elapsed_ms, arrays["frontier"][:k].copy(),
                 arrays["edges"][:k].copy(), arrays["scatter_ms"][:k].copy() if timing else None,
                 arrays["step_ms"][:k].copy() if timing else None, arrays["schedule"][:k].copy())


class Batch:
    """Many CC / SSSP queries over many graphs in one run (vc_batch_*).

    members: list of rmatgen.Csr (host) or (offsets, dst, weights) CUDA
    tensor triples; queries: list of ("cc" | "sssp", source).  The library
    copies the members into one device-resident union.
    """

    def __init__(self, members, queries, *, validate: bool = False, relabel: bool = True, stream=None, device=None):
        import torch
        lib = load()
        if len(members) != len(queries) or not members:
            raise ValueError("members and queries must be non-empty and of equal length")
        device = torch.device("cuda", torch.cuda.current_device()) if device is None else device
        keep = []
        descs = (GraphDesc * len(members))()
        qs = (BatchQuery * len(members))()
        for i, (mem, (prog, src)) in enumerate(zip(members, queries)):
            if isinstance(mem, tuple):
                off, dst, w = mem
            else:
                off = torch.from_numpy(np.ascontiguousarray(mem.off)).to(device)
                dst = torch.from_numpy(np.ascontiguousarray(mem.dst)).to(device)
                w = None if mem.w is None else torch.from_numpy(np.ascontiguousarray(mem.w).view(np.int32)).to(device)
            keep.append((off, dst, w))
            n, m = off.numel() - 1, dst.numel()
            descs[i] = GraphDesc(ctypes.sizeof(GraphDesc), 0, n, m,
                                 IDX_I64 if off.dtype == torch.int64 else IDX_I32, off.data_ptr(),
                                 dst.data_ptr() if m else None, w.data_ptr() if (w is not None and m) else None)
            qs[i] = BatchQuery(ctypes.sizeof(BatchQuery), _program(prog), int(src))
        torch.cuda.synchronize(device)
        h = ctypes.c_void_p()
        flags = (GRAPH_VALIDATE if validate else 0) | (0 if relabel else GRAPH_NO_RELABEL)
        _check(lib.vc_batch_create(descs, qs, len(members), flags, _stream_handle(stream), ctypes.byref(h)),
               "vc_batch_create")
        self._h = h
        self.count = len(members)
        base = np.zeros(self.count + 1, np.int64)
        _check(lib.vc_batch_layout(h, base.ctypes.data), "vc_batch_layout")
        self.vertex_base = base
        self.n = int(base[-1])
        self.device = device

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().vc_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune(self, stream=None) -> dict:
        """vc_batch_autotune: picks and keeps the fastest distribution for the batch."""
        base = _params(0, 0.85, 0, "auto", 0, 0)
        best = Params()
        _check(load().vc_batch_autotune(self._h, ctypes.byref(base), _stream_handle(stream), ctypes.byref(best)),
               "vc_batch_autotune")
        return _params_dict(best)

    def run(self, out=None, *, max_supersteps: int = 0, schedule="auto", tile: int = 0, options: int = 0,
            pull_fraction: float = 0.0, stream=None, stats: bool = False, timing: bool = False,
            capacity: int = 4096):
        import torch
        if out is None:
            out = torch.empty(self.n, dtype=torch.int32, device=self.device)
        if not out.is_cuda or not out.is_contiguous() or out.numel() != self.n or out.element_size() != 4:
            raise TypeError("out must be a contiguous CUDA tensor of sum(N_i) 4-byte elements")
        p = _params(max_supersteps, 0.85, 0, schedule, tile, options, pull_fraction)
        st, arrays = _stats_struct(stats or timing, timing, capacity)
        rc = load().vc_batch_run(self._h, ctypes.byref(p), out.data_ptr(), _stream_handle(stream),
                                 ctypes.byref(st) if st is not None else None)
        _check(rc, "vc_batch_run")
        return out, _stats_result(st, arrays, capacity)

    def split(self, out):
        """Host numpy uint32 results, one array per member."""
        vals = out.cpu().numpy().view(np.uint32)
        return [vals[self.vertex_base[i]:self.vertex_base[i + 1]] for i in range(self.count)]


@dataclass
class Completion:
    ticket: int
    tag: int
    status: int
    supersteps: int
    lane: int
    queue_ms: float
    service_ms: float
    message: str

    @property
    def latency_ms(self) -> float:
        return self.queue_ms + self.service_ms


class Server:
    """Request server over resident graphs (vc_server_*).

    Graphs are registered with add_graph (lanes > 0 gives the graph a lane
    table for continuous batching of CC / SSSP requests); submit queues one
    request and returns its ticket; poll / drain collect completions.  A
    request's `out` tensor is referenced until its completion is polled.
    """

    def __init__(self, *, workers: int = 2, hbm_budget: int = 0, device=None):
        import torch
        lib = load()
        cfg = ServerConfig(ctypes.sizeof(ServerConfig), int(workers), int(hbm_budget))
        h = ctypes.c_void_p()
        _check(lib.vc_server_create(ctypes.byref(cfg), ctypes.byref(h)), "vc_server_create")
        self._h = h
        self._graphs = []
        self._pending = {}
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else device

    def add_graph(self, graph: Graph, lanes: int = 0, rank_lanes: int = 0) -> int:
        gid = ctypes.c_int32()
        _check(load().vc_server_add_graph(self._h, graph._h, int(lanes), int(rank_lanes), ctypes.byref(gid)),
               "vc_server_add_graph")
        self._graphs.append(graph)
        return gid.value

    def submit(self, graph_id: int, program, out, *, source: int = 0, T: int = 10, damping: float = 0.85,
               max_supersteps: int = 0, schedule="auto", tile: int = 0, options: int = 0, tag: int = 0,
               route="auto") -> int:
        prog = _program(program)
        rank = prog in (PAGERANK, PPR)
        if not out.is_cuda or not out.is_contiguous() or out.element_size() != 4:
            raise TypeError("out must be a contiguous CUDA tensor of 4-byte elements")
        n = self._graphs[graph_id].n if 0 <= graph_id < len(self._graphs) else None
        if n is not None and out.numel() != n:
            raise TypeError("out must hold N elements")
        req = Request(ctypes.sizeof(Request), int(graph_id), prog, ROUTES[route] if isinstance(route, str) else int(route),
                      _params(T if rank else max_supersteps, damping, source, schedule, tile, options),
                      out.data_ptr(), int(tag))
        ticket = ctypes.c_uint64()
        _check(load().vc_server_submit(self._h, ctypes.byref(req), ctypes.byref(ticket)), "vc_server_submit")
        self._pending[ticket.value] = out
        return ticket.value

    def poll(self, timeout_ms: int = 0, cap: int = 256):
        buf = (CompletionStruct * cap)()
        k = ctypes.c_int32()
        _check(load().vc_server_poll(self._h, buf, cap, int(timeout_ms), ctypes.byref(k)), "vc_server_poll")
        res = []
        for c in buf[:k.value]:
            self._pending.pop(c.ticket, None)
            res.append(Completion(c.ticket, c.tag, c.status, c.supersteps, c.lane, c.queue_ms, c.service_ms,
                                  c.message.decode(errors="replace")))
        return res

    def drain(self):
        _check(load().vc_server_drain(self._h), "vc_server_drain")

    def info(self) -> dict:
        st = ServerInfo()
        st.struct_size = ctypes.sizeof(ServerInfo)
        _check(load().vc_server_info_get(self._h, ctypes.byref(st)), "vc_server_info_get")
        return {f: getattr(st, f) for f, _ in ServerInfo._fields_ if f != "struct_size"}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().vc_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._pending.clear()
            self._graphs = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
