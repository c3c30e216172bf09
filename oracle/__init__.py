"""CPU oracle of the Pregel superstep -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The GPU library never loads it,
and it shares no code with the GPU library.

``run(program, csr, ...)`` executes the plain sequential C engine in
``oracle.c`` (paper, Section I execution model; Section III mailboxes with
explicit flags; Section VI-C benchmark programs) and returns the final values
(float64 ranks, or uint32 labels / distances) and per-superstep statistics.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_DIR = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_DIR, "oracle.c")
_LIB = os.path.join(_DIR, "liboracle.so")
_lib = None

PAGERANK, CC, SSSP, PPR = 0, 1, 2, 3
PROGRAMS = {"pagerank": PAGERANK, "cc": CC, "sssp": SSSP, "ppr": PPR}
UNREACHED = 0xFFFFFFFF
_ERRORS = {-1: "invalid argument", -2: "out of memory", -3: "distance overflows uint32", -4: "superstep cap reached"}


class OracleError(RuntimeError):
    pass


def build() -> None:
    """Compiles the oracle (plain C11, one thread)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-fPIC", "-shared", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)


class _Step(ctypes.Structure):
    _fields_ = [("senders", ctypes.c_int64), ("messages", ctypes.c_int64), ("receivers", ctypes.c_int64)]


def _bind(path):
    lib = ctypes.CDLL(path)
    i64, i32, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
    lib.oracle_run.restype = ctypes.c_int
    lib.oracle_run.argtypes = [ctypes.c_int, i64, vp, vp, vp, i32, ctypes.c_double, i64, i64, vp, vp, i64,
                               ctypes.POINTER(i64)]
    lib.oracle_version.restype = ctypes.c_int
    lib.oracle_combine.restype = ctypes.c_int
    lib.oracle_combine.argtypes = [ctypes.c_int, i64, vp, vp, vp, vp, vp, vp]
    return lib


VERSION = 2


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(_LIB)
        if _lib.oracle_version() != VERSION:
            raise OracleError(f"{_LIB} is a stale build; delete it and rebuild")
    return _lib


def load_variant(path):
    """Binds another build of the oracle source (used by the mutation tests)."""
    return _bind(path)


@dataclass
class Result:
    values: np.ndarray  # float64 ranks, or uint32 labels / distances
    supersteps: int
    senders: np.ndarray  # |F_s|
    messages: np.ndarray  # E_s
    receivers: np.ndarray  # |R_s|


def run(program, n, off, dst, w=None, T: int = 10, damping: float = 0.85, source: int = 0,
        max_supersteps: int = 0, lib=None) -> Result:
    """Runs `program` ("pagerank", "cc", "sssp", "ppr") on the CSR (off, dst, w)."""
    lib = _load() if lib is None else lib
    prog = PROGRAMS[program] if isinstance(program, str) else int(program)
    off64 = np.ascontiguousarray(off, dtype=np.int64)
    dst32 = np.ascontiguousarray(dst, dtype=np.int32)
    w32 = None if w is None else np.ascontiguousarray(w, dtype=np.uint32)
    if off64.shape[0] != n + 1 or dst32.shape[0] != off64[-1]:
        raise ValueError("CSR arrays do not match n")
    is_rank = prog in (PAGERANK, PPR)
    out = np.empty(n, dtype=np.float64 if is_rank else np.uint32)
    cap = (T + 2) if is_rank else min(max_supersteps if max_supersteps > 0 else n + 2, 1 << 16)
    cap = max(int(cap), 1)
    steps = (_Step * cap)()
    nsteps = ctypes.c_int64(0)
    rc = lib.oracle_run(prog, int(n), off64.ctypes.data, dst32.ctypes.data if dst32.size else None,
                        None if w32 is None else w32.ctypes.data, int(T), float(damping), int(source),
                        int(max_supersteps), out.ctypes.data, steps, cap, ctypes.byref(nsteps))
    if rc != 0:
        raise OracleError(_ERRORS.get(rc, f"error {rc}"))
    k = min(int(nsteps.value), cap)
    arr = np.frombuffer(steps, dtype=np.int64).reshape(cap, 3)[:k].copy()
    return Result(out, int(nsteps.value), arr[:, 0], arr[:, 1], arr[:, 2])


COMBINERS = {"sum_u64": 0, "prod_u64": 1, "max_f64": 2, "minarg": 3, "sum_f64": 4}


def combine(op, n, off, dst, msg, active=None, lib=None):
    """One superstep of message passing with combiner `op` (see COMBINERS):
    every active vertex sends its 8-byte message msg[v] along its out-edges.
    Returns (mailbox uint64 words, has-message flags as bool)."""
    lib = _load() if lib is None else lib
    code = COMBINERS[op] if isinstance(op, str) else int(op)
    off64 = np.ascontiguousarray(off, dtype=np.int64)
    dst32 = np.ascontiguousarray(dst, dtype=np.int32)
    words = np.ascontiguousarray(np.asarray(msg).view(np.uint64) if np.asarray(msg).dtype != np.uint64 else msg,
                                 dtype=np.uint64)
    if off64.shape[0] != n + 1 or words.shape[0] != n:
        raise ValueError("arrays do not match n")
    act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
    box = np.empty(n, np.uint64)
    has = np.empty(n, np.uint8)
    rc = lib.oracle_combine(code, int(n), off64.ctypes.data, dst32.ctypes.data if dst32.size else None,
                            words.ctypes.data, None if act is None else act.ctypes.data, box.ctypes.data,
                            has.ctypes.data)
    if rc != 0:
        raise OracleError(_ERRORS.get(rc, f"error {rc}"))
    return box, has.astype(bool)


def run_csr(program, g, **kw) -> Result:
    """`run` on an ``rmatgen.Csr``."""
    return run(program, g.n, g.off, g.dst, g.w, **kw)
