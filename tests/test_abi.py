"""The C-ABI library loads and exports every symbol the header declares (no GPU calls)."""
import ctypes
import os
import subprocess

import pytest

from paper_2305_17813_amd import native


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(native.LIB_PATH):
        from paper_2305_17813_amd import build
        build.build()
    return native.LIB_PATH


def test_header_declares_the_boundary():
    names = native.declared_symbols()
    for must in ["mk_arena_bytes", "mk_graph_create", "mk_graph_destroy", "mk_insert_edges",
                 "mk_delete_edges", "mk_query_edges", "mk_incr_bfs", "mk_incr_sssp", "mk_incr_wcc",
                 "mk_incr_pagerank", "mk_count_triangles", "mk_graph_export", "mk_graph_stats",
                 "mk_graph_check", "mk_status_string"]:
        assert must in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    for name in native.declared_symbols():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lib_path], capture_output=True, text=True).stdout
    for name in native.declared_symbols():
        assert f" T {name}" in out, name


def test_status_strings_without_gpu(lib_path):
    lib = native.load()
    assert lib.mk_status_string(0) == b"ok"
    assert b"nothing applied" in lib.mk_status_string(2)


def test_null_arguments_rejected_without_gpu(lib_path):
    lib = native.load()
    assert lib.mk_graph_destroy(None) == 0
    assert lib.mk_insert_edges(None, None, None, None, 1, None, None) == 1
    assert lib.mk_query_edges(None, None, None, 1, None, None, None) == 1
    assert lib.mk_set_iteration_scheme(None, 2) == 1
    assert lib.mk_set_cost_model(None, None) == 1
    cfg = native.MkConfig(0, 1, 0.7, 1, 0, 0)
    h = ctypes.c_void_p()
    assert lib.mk_graph_create(ctypes.byref(cfg), None, 0, None, None, None, 0, None, ctypes.byref(h)) == 1
