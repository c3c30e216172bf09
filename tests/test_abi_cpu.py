"""The C ABI library on the CPU: it loads, exports every declared symbol, and
rejects bad arguments before touching the device (no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2010_01542_amd import vc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*(vc_[a-z_]+)\s*\(", text,
                                 flags=re.M)))


def test_header_declares_the_binding_exports():
    assert sorted(vc.EXPORTS) == declared_functions()


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(vc.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_abi_version_and_status_strings():
    lib = vc.load()
    assert lib.vc_abi_version() == vc.ABI_VERSION
    for s in range(7):
        assert lib.vc_status_string(s)
    assert lib.vc_status_string(99) == b"unknown status"


def test_params_default():
    lib = vc.load()
    p = vc.Params()
    lib.vc_params_default(ctypes.byref(p))
    assert p.struct_size == ctypes.sizeof(vc.Params)
    assert p.max_supersteps == 10 and p.damping == pytest.approx(0.85) and p.schedule == vc.SCHED_AUTO


def test_struct_layout_matches_header(tmp_path):
    """sizeof / offsetof of every ABI struct field, from the C compiler, equal ctypes'."""
    structs = {"vc_graph_desc": vc.GraphDesc, "vc_params": vc.Params, "vc_stats": vc.StatsStruct,
               "vc_batch_query": vc.BatchQuery, "vc_server_config": vc.ServerConfig, "vc_request": vc.Request,
               "vc_completion": vc.CompletionStruct, "vc_server_info": vc.ServerInfo}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "vc.h"', "int main(void) {"]
    for cname, cls in structs.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I",
                           "/opt/rocm/include", "-o", str(exe), str(src)])
    got = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for cname, cls in structs.items():
        assert int(got[f"{cname} sizeof"]) == ctypes.sizeof(cls)
        for fname, _ in cls._fields_:
            assert int(got[f"{cname} {fname}"]) == getattr(cls, fname).offset, (cname, fname)


def test_enum_values_match_header(tmp_path):
    """Every enumerator the binding mirrors has the header's value."""
    names = {
        "VC_OK": vc.OK, "VC_ERR_INVALID_ARG": vc.ERR_INVALID_ARG, "VC_ERR_BAD_GRAPH": vc.ERR_BAD_GRAPH,
        "VC_ERR_OUT_OF_MEMORY": vc.ERR_OUT_OF_MEMORY, "VC_ERR_HIP": vc.ERR_HIP,
        "VC_ERR_UNSUPPORTED": vc.ERR_UNSUPPORTED, "VC_ERR_NOT_CONVERGED": vc.ERR_NOT_CONVERGED,
        "VC_PAGERANK": vc.PAGERANK, "VC_CC_HASHMIN": vc.CC_HASHMIN, "VC_SSSP": vc.SSSP, "VC_PPR": vc.PPR,
        "VC_SCHED_AUTO": vc.SCHED_AUTO, "VC_SCHED_VERTEX": vc.SCHED_VERTEX, "VC_SCHED_EDGE": vc.SCHED_EDGE,
        "VC_SCHED_PULL": vc.SCHED_PULL, "VC_SCHED_BLOCKED": vc.SCHED_BLOCKED,
        "VC_OPT_NO_HUB_AGGREGATION": vc.OPT_NO_HUB_AGGREGATION,
        "VC_OPT_NO_TEST_BEFORE_ATOMIC": vc.OPT_NO_TEST_BEFORE_ATOMIC,
        "VC_OPT_F32_ACCUMULATE": vc.OPT_F32_ACCUMULATE, "VC_OPT_GRAPH_CAPTURE": vc.OPT_GRAPH_CAPTURE,
        "VC_OPT_F32_MESSAGES": vc.OPT_F32_MESSAGES,
        "VC_ROUTE_AUTO": vc.ROUTE_AUTO, "VC_ROUTE_LANES": vc.ROUTE_LANES, "VC_ROUTE_WORKER": vc.ROUTE_WORKER,
    }
    names.update({f"VC_COMBINE_{k.upper()}": v for k, v in vc.COMBINERS.items()})
    lines = ["#include <stdio.h>", '#include "vc.h"', "int main(void) {"]
    lines += [f'printf("{k} %ld\\n", (long){k});' for k in names]
    lines.append("return 0; }")
    src = tmp_path / "enums.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "enums"
    subprocess.check_call(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-I",
                           "/opt/rocm/include", "-o", str(exe), str(src)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)], text=True).splitlines())
    for k, v in names.items():
        assert int(got[k]) == v, k


def test_argument_errors_need_no_device():
    lib = vc.load()
    h = ctypes.c_void_p()
    assert lib.vc_graph_create(None, None, ctypes.byref(h)) == vc.ERR_INVALID_ARG
    d = vc.GraphDesc(ctypes.sizeof(vc.GraphDesc) + 1, 0, 4, 0, vc.IDX_I32, 8, 8, None)
    assert lib.vc_graph_create(ctypes.byref(d), None, ctypes.byref(h)) == vc.ERR_INVALID_ARG
    assert b"struct_size" in lib.vc_last_error()
    d = vc.GraphDesc(ctypes.sizeof(vc.GraphDesc), 0, 0, 0, vc.IDX_I32, 8, 8, None)
    assert lib.vc_graph_create(ctypes.byref(d), None, ctypes.byref(h)) == vc.ERR_INVALID_ARG
    d = vc.GraphDesc(ctypes.sizeof(vc.GraphDesc), 0, 4, 2**31, vc.IDX_I32, 8, 8, None)
    assert lib.vc_graph_create(ctypes.byref(d), None, ctypes.byref(h)) == vc.ERR_INVALID_ARG
    assert b"int32 offsets" in lib.vc_last_error()
    d = vc.GraphDesc(ctypes.sizeof(vc.GraphDesc), 0, 4, 3, vc.IDX_I64, 12, 8, None)
    assert lib.vc_graph_create(ctypes.byref(d), None, ctypes.byref(h)) == vc.ERR_INVALID_ARG
    assert b"misaligned" in lib.vc_last_error()
    assert lib.vc_run(None, vc.SSSP, None, 16, None, None) == vc.ERR_INVALID_ARG
    assert lib.vc_graph_prepare(None, vc.SSSP, None, None) == vc.ERR_INVALID_ARG
    assert lib.vc_graph_destroy(None) == vc.OK
    held = ctypes.c_size_t()
    assert lib.vc_graph_footprint(None, 0, ctypes.byref(held), None) == vc.ERR_INVALID_ARG
    b = ctypes.c_void_p()
    assert lib.vc_batch_create(None, None, 0, 0, None, ctypes.byref(b)) == vc.ERR_INVALID_ARG
    descs = (vc.GraphDesc * 1)(vc.GraphDesc(ctypes.sizeof(vc.GraphDesc), 0, 4, 0, vc.IDX_I32, 8, 8, None))
    qs = (vc.BatchQuery * 1)(vc.BatchQuery(ctypes.sizeof(vc.BatchQuery), vc.PAGERANK, 0))
    assert lib.vc_batch_create(descs, qs, 1, 0, None, ctypes.byref(b)) == vc.ERR_UNSUPPORTED
    qs[0] = vc.BatchQuery(ctypes.sizeof(vc.BatchQuery), vc.SSSP, 4)
    assert lib.vc_batch_create(descs, qs, 1, 0, None, ctypes.byref(b)) == vc.ERR_INVALID_ARG
    assert lib.vc_batch_run(None, None, 16, None, None) == vc.ERR_INVALID_ARG
    assert lib.vc_batch_destroy(None) == vc.OK
    # request server
    srv = ctypes.c_void_p()
    assert lib.vc_server_create(None, None) == vc.ERR_INVALID_ARG
    cfg = vc.ServerConfig(ctypes.sizeof(vc.ServerConfig) - 8, 2, 0)
    assert lib.vc_server_create(ctypes.byref(cfg), ctypes.byref(srv)) == vc.ERR_INVALID_ARG
    cfg = vc.ServerConfig(ctypes.sizeof(vc.ServerConfig), 65, 0)
    assert lib.vc_server_create(ctypes.byref(cfg), ctypes.byref(srv)) == vc.ERR_INVALID_ARG
    assert b"workers" in lib.vc_last_error()
    gid = ctypes.c_int32()
    assert lib.vc_server_add_graph(None, None, 64, 0, ctypes.byref(gid)) == vc.ERR_INVALID_ARG
    assert lib.vc_server_submit(None, None, None) == vc.ERR_INVALID_ARG
    cnt = ctypes.c_int32()
    assert lib.vc_server_poll(None, None, 0, 0, ctypes.byref(cnt)) == vc.ERR_INVALID_ARG
    assert lib.vc_server_drain(None) == vc.ERR_INVALID_ARG
    assert lib.vc_server_info_get(None, None) == vc.ERR_INVALID_ARG
    assert lib.vc_server_destroy(None) == vc.OK
