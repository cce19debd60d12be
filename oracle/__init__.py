"""CPU oracle (test infrastructure only).

A plain, single-threaded C++ reference of what the GPU path computes: sorted adjacency
sets, insert/delete/search by their set semantics, and every algorithm recomputed from
scratch after each batch (queue BFS, Dijkstra, union-find, FP64 power-iteration
PageRank, oriented sorted-list triangle counting).  Only ``tests/``, the smoke entry
point and the benchmark's CPU-baseline leg may use it; the product path never does.

Parity unpinned: nothing here -- every function is pinned by the "not gpu" tests
(closed forms, brute force on tiny graphs, independent textbook methods).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

U32P = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
U8P = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
F64P = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (single-threaded, -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp, u32, u64 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64
        L.orc_create.restype = vp
        L.orc_create.argtypes = [u32, U32P, U32P, ctypes.c_void_p, u64]
        L.orc_destroy.argtypes = [vp]
        L.orc_num_arcs.restype = u64
        L.orc_num_arcs.argtypes = [vp]
        L.orc_out_degree.argtypes = [vp, U32P]
        L.orc_undirected_degree.argtypes = [vp, U32P]
        L.orc_insert.argtypes = [vp, U32P, U32P, ctypes.c_void_p, u64, U8P]
        L.orc_delete.argtypes = [vp, U32P, U32P, u64, U8P]
        L.orc_query.argtypes = [vp, U32P, U32P, u64, U8P, U32P]
        L.orc_export.restype = u64
        L.orc_export.argtypes = [vp, U32P, U32P, U32P]
        L.orc_bfs.argtypes = [vp, u32, U32P, U32P]
        L.orc_sssp.restype = ctypes.c_int
        L.orc_sssp.argtypes = [vp, u32, U32P, U32P]
        L.orc_wcc.argtypes = [vp, U32P]
        L.orc_pagerank.restype = u32
        L.orc_pagerank.argtypes = [vp, ctypes.c_double, ctypes.c_double, u32, ctypes.c_int, F64P]
        L.orc_triangles.restype = u64
        L.orc_triangles.argtypes = [vp]
        L.orc_triangles_brute.restype = u64
        L.orc_triangles_brute.argtypes = [vp]
        L.orc_triangles_touching.restype = u64
        L.orc_triangles_touching.argtypes = [vp, U32P, U32P, u64]
        _lib = L
    return _lib


def _u32(a) -> np.ndarray:
    if hasattr(a, "cpu"):
        a = a.cpu().numpy()
    a = np.asarray(a)
    if a.dtype == np.int32:
        a = a.view(np.uint32)
    return np.ascontiguousarray(a.astype(np.uint32, copy=False))


INF = 0xFFFFFFFF
NO_VERTEX = 0xFFFFFFFF


class OracleGraph:
    """Sorted-adjacency reference graph; every query recomputes from scratch."""

    def __init__(self, n: int, src, dst, w=None):
        L = lib()
        self.n = int(n)
        s, d = _u32(src), _u32(dst)
        self._w = None if w is None else _u32(w)
        wp = None if self._w is None else self._w.ctypes.data_as(ctypes.c_void_p)
        self.h = L.orc_create(self.n, s, d, wp, s.size)

    def close(self):
        if self.h:
            lib().orc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def m(self) -> int:
        return int(lib().orc_num_arcs(self.h))

    def out_degree(self) -> np.ndarray:
        d = np.zeros(self.n, np.uint32)
        lib().orc_out_degree(self.h, d)
        return d

    def undirected_degree(self) -> np.ndarray:
        d = np.zeros(self.n, np.uint32)
        lib().orc_undirected_degree(self.h, d)
        return d

    def insert(self, src, dst, w=None) -> np.ndarray:
        s, d = _u32(src), _u32(dst)
        ww = None if w is None else _u32(w)
        st = np.zeros(s.size, np.uint8)
        lib().orc_insert(self.h, s, d, None if ww is None else ww.ctypes.data_as(ctypes.c_void_p),
                         s.size, st)
        return st

    def delete(self, src, dst) -> np.ndarray:
        s, d = _u32(src), _u32(dst)
        st = np.zeros(s.size, np.uint8)
        lib().orc_delete(self.h, s, d, s.size, st)
        return st

    def query(self, src, dst):
        s, d = _u32(src), _u32(dst)
        f = np.zeros(s.size, np.uint8)
        w = np.zeros(s.size, np.uint32)
        lib().orc_query(self.h, s, d, s.size, f, w)
        return f, w

    def export(self):
        m = self.m
        s = np.zeros(m, np.uint32)
        d = np.zeros(m, np.uint32)
        w = np.zeros(m, np.uint32)
        lib().orc_export(self.h, s, d, w)
        return s, d, w

    def bfs(self, source: int):
        lv = np.zeros(self.n, np.uint32)
        pa = np.zeros(self.n, np.uint32)
        lib().orc_bfs(self.h, int(source), lv, pa)
        return lv, pa

    def sssp(self, source: int):
        di = np.zeros(self.n, np.uint32)
        pa = np.zeros(self.n, np.uint32)
        ov = lib().orc_sssp(self.h, int(source), di, pa)
        assert ov == 0, "a shortest distance does not fit in 32 bits"
        return di, pa

    def wcc(self) -> np.ndarray:
        lab = np.zeros(self.n, np.uint32)
        lib().orc_wcc(self.h, lab)
        return lab

    def pagerank(self, damping=0.85, tol=1e-13, max_iter=10000, warm=None):
        r = np.zeros(self.n, np.float64) if warm is None else np.ascontiguousarray(warm, np.float64)
        it = lib().orc_pagerank(self.h, float(damping), float(tol), int(max_iter),
                                0 if warm is None else 1, r)
        return r, int(it)

    def triangles(self) -> int:
        return int(lib().orc_triangles(self.h))

    def triangles_brute(self) -> int:
        return int(lib().orc_triangles_brute(self.h))

    def triangles_touching(self, a, b) -> int:
        """Triangles of the underlying undirected graph with at least one edge among the
        pairs {a[i], b[i]} (each counted once)."""
        x, y = _u32(a), _u32(b)
        return int(lib().orc_triangles_touching(self.h, x, y, x.size))
