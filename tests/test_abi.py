"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/n2vwalk.h, and rejects bad arguments
before touching the device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "n2vwalk.h")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(n2v_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["n2v_graph_upload", "n2v_graph_info", "n2v_graph_release", "n2v_walks_first_order",
                 "n2v_walks_node2vec", "n2v_walks_batched", "n2v_server_create", "n2v_request_submit",
                 "n2v_request_poll", "n2v_request_release", "n2v_server_destroy", "n2v_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2110_06196_amd as n2v
    L = n2v.lib()
    for name in declared():
        assert hasattr(L, name), name
        assert name in n2v.SIGNATURES, name
    out = subprocess.run(["nm", "-D", "--defined-only", n2v.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (n2v_\w+)", out))
    assert set(declared()) <= exported


def test_argument_validation_without_device():
    import paper_2110_06196_amd as n2v
    L = n2v.lib()
    h = ctypes.c_uint64(7)
    assert L.n2v_graph_upload(None, 0, None, 0, None, 0, None, ctypes.byref(h)) == n2v.N2V_ERR_INVALID_ARG
    assert h.value == 0
    assert b"offsets" in L.n2v_last_error()
    assert L.n2v_graph_upload(ctypes.c_void_p(8), 1, None, 5, None, 0, None, ctypes.byref(h)) == n2v.N2V_ERR_INVALID_ARG
    assert L.n2v_graph_upload(ctypes.c_void_p(8), 1, ctypes.c_void_p(8), 1, None, 4, None, ctypes.byref(h)) == n2v.N2V_ERR_INVALID_ARG
    assert L.n2v_graph_upload(ctypes.c_void_p(8), 1, ctypes.c_void_p(8), 1, None, 1 << 13, None, ctypes.byref(h)) == n2v.N2V_ERR_INVALID_ARG
    assert L.n2v_graph_upload(ctypes.c_void_p(8), 2**31, ctypes.c_void_p(8), 1, None, 0, None, ctypes.byref(h)) == n2v.N2V_ERR_INVALID_ARG
    assert L.n2v_walks_first_order(12345, None, 0, 1, 1, 0, 0, None, None, None) == n2v.N2V_ERR_BAD_HANDLE
    assert L.n2v_walks_node2vec(12345, None, 0, 1, 1, 1.0, 1.0, 0, 0, None, None, None) == n2v.N2V_ERR_BAD_HANDLE
    assert L.n2v_graph_release(999) == n2v.N2V_ERR_BAD_HANDLE
    info = n2v.GraphInfo()
    assert L.n2v_graph_info(999, ctypes.byref(info)) == n2v.N2V_ERR_BAD_HANDLE
    bad = n2v.Tuning(7, 0, 0, 0, 0)
    assert L.n2v_set_tuning(ctypes.byref(bad)) == n2v.N2V_ERR_INVALID_ARG
    bad = n2v.Tuning(16, 0, 0, 9, 0)
    assert L.n2v_set_tuning(ctypes.byref(bad)) == n2v.N2V_ERR_INVALID_ARG
    assert L.n2v_set_tuning(None) == n2v.N2V_OK
    # a server's own tuning is checked like n2v_set_tuning's, before any device call
    bad = n2v.Tuning(7, 0, 0, 0, 0)
    assert L.n2v_server_create(1 << 20, 4, ctypes.byref(bad), ctypes.byref(h)) == n2v.N2V_ERR_INVALID_ARG
    assert h.value == 0 and b"lanes_per_walker" in L.n2v_last_error()
    bad = n2v.Tuning(16, 0, 0, 0, 8)
    assert L.n2v_server_create(1 << 20, 4, ctypes.byref(bad), ctypes.byref(h)) == n2v.N2V_ERR_INVALID_ARG
    assert L.n2v_walks_batched(None, 3, None) == n2v.N2V_ERR_INVALID_ARG
    # the allocation-free batched form: NULL table and its request limit
    assert L.n2v_walks_batched_noalloc(None, 3, None) == n2v.N2V_ERR_INVALID_ARG
    over = (n2v.RequestDesc * 4097)()
    assert L.n2v_walks_batched_noalloc(over, 4097, None) == n2v.N2V_ERR_INVALID_ARG
    assert b"4096" in L.n2v_last_error()
    # Elias-Fano graphs: argument checks come before any device call
    assert L.n2v_graph_upload_ef(None, 1, None, 0, None, 0, None, ctypes.byref(h)) == n2v.N2V_ERR_INVALID_ARG
    assert L.n2v_graph_upload_ef(ctypes.c_void_p(8), 0, None, 0, None, 0, None, ctypes.byref(h)) == n2v.N2V_ERR_INVALID_ARG
    for q in (4, 7, 100, 1 << 17):
        assert L.n2v_graph_upload_ef(ctypes.c_void_p(8), 1, None, 0, None, q, None, ctypes.byref(h)) == n2v.N2V_ERR_INVALID_ARG
    ef = n2v.EFInfo()
    assert L.n2v_ef_info(999, ctypes.byref(ef)) == n2v.N2V_ERR_BAD_HANDLE
    assert L.n2v_ef_select(999, None, 0, None, None) == n2v.N2V_ERR_BAD_HANDLE
    assert L.n2v_ef_rank(999, None, 0, None, None) == n2v.N2V_ERR_BAD_HANDLE


def test_product_has_no_oracle_dependency():
    """The GPU package never imports or links the oracle."""
    pkg = os.path.join(ROOT, "paper_2110_06196_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                txt = open(os.path.join(dp, f)).read()
                assert "oracle" not in txt.replace("oracle-free", ""), f
