"""Thin ctypes binding of libmeerkat_mi355x.so: argument marshalling only.

Every step of the path runs in the HIP library; this module only turns torch tensors
(device memory, streams) into the pointers and sizes the C-ABI takes, and raises on a
non-OK status.  It fails loudly when the library has not been built: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmeerkat_mi355x.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "meerkat_mi355x.h")

VIEW_FWD, VIEW_REV, VIEW_UND = 1, 2, 4
AUTO, INCR, RECOMPUTE = 0, 1, 2
# incremental-WCC schemes (mk_wcc_scheme)
WCC_LOG, WCC_NAIVE, WCC_SLAB, WCC_UPDATE = 0, 1, 2, 3
# iteration schemes of all-vertex walks (mk_iter_scheme)
ITER_SCHEME1, ITER_SCHEME2, ITER_PACKED = 1, 2, 3
STATUS_NAMES = {0: "MK_OK", 1: "MK_ERR_INVALID_ARG", 2: "MK_ERR_OUT_OF_SLABS", 3: "MK_ERR_CAPACITY",
                4: "MK_ERR_STATE", 5: "MK_ERR_HIP"}


class MkError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}")
        self.status = status


class MkConfig(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_uint32), ("views", ctypes.c_uint32),
                ("load_factor", ctypes.c_float), ("hash_seed", ctypes.c_uint32),
                ("pool_slabs", ctypes.c_uint64), ("log_capacity", ctypes.c_uint64),
                ("sssp_delta", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class MkStats(ctypes.Structure):
    _fields_ = [("n_arcs", ctypes.c_uint64), ("n_und_edges", ctypes.c_uint64),
                ("head_slabs", ctypes.c_uint64 * 3), ("pool_used", ctypes.c_uint64 * 3),
                ("pool_capacity", ctypes.c_uint64 * 3), ("arena_bytes_used", ctypes.c_uint64),
                ("batches_applied", ctypes.c_uint64)]

    def as_dict(self):
        return {"n_arcs": self.n_arcs, "n_und_edges": self.n_und_edges,
                "head_slabs": list(self.head_slabs), "pool_used": list(self.pool_used),
                "pool_capacity": list(self.pool_capacity),
                "arena_bytes_used": self.arena_bytes_used,
                "batches_applied": self.batches_applied}


_lib = None


def declared_symbols():
    """Names of the functions the C-ABI header declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(mk_\w+)\s*\(", text, re.M)))


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                           "(run __graft_entry__.build() or python paper_2305_17813_amd/build.py)")
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    L.mk_arena_bytes.restype = ctypes.c_size_t
    L.mk_arena_bytes.argtypes = [ctypes.POINTER(MkConfig), u64]
    sigs = {
        "mk_graph_create": [ctypes.POINTER(MkConfig), vp, ctypes.c_size_t, vp, vp, vp, u64, vp,
                            ctypes.POINTER(vp)],
        "mk_graph_destroy": [vp],
        "mk_insert_edges": [vp, vp, vp, vp, u64, vp, vp],
        "mk_delete_edges": [vp, vp, vp, u64, vp, vp],
        "mk_query_edges": [vp, vp, vp, u64, vp, vp, vp],
        "mk_incr_bfs": [vp, u32, vp, vp, i32, vp],
        "mk_incr_sssp": [vp, u32, vp, vp, i32, vp],
        "mk_incr_wcc": [vp, vp, i32, vp],
        "mk_incr_wcc_scheme": [vp, vp, i32, i32, vp],
        "mk_incr_pagerank": [vp, ctypes.c_float, ctypes.c_double, u32, vp, vp, i32, vp],
        "mk_count_triangles": [vp, vp, i32, vp],
        "mk_graph_export": [vp, vp, vp, vp, u64, ctypes.POINTER(u64), vp],
        "mk_graph_stats": [vp, ctypes.POINTER(MkStats), vp],
        "mk_graph_check": [vp, ctypes.POINTER(u64), vp],
        "mk_probe_cost": [vp, i32, i32, vp, vp, u64, ctypes.POINTER(u64), vp],
        "mk_compact": [vp, u32, ctypes.POINTER(u64), vp],
        "mk_batch_features": [vp, i32, vp, vp, vp, u64, vp, vp, u64, ctypes.POINTER(ctypes.c_float), vp],
        "mk_mlp_forward": [vp, vp, u32, vp, vp],
        "mk_traverse_from": [vp, u32, i32, vp, ctypes.c_size_t, u32, vp, vp, vp],
        "mk_bfs_levels": [vp, u32, u32, vp, ctypes.c_size_t, u32, vp, ctypes.POINTER(u32), vp],
        "mk_sssp_distances": [vp, u32, vp, ctypes.c_size_t, u32, vp, vp],
        "mk_mlp_grad": [vp, vp, vp, vp, u32, vp, vp, ctypes.c_size_t, vp, vp],
        "mk_mlp_grad_static": [vp, vp, vp, vp, u32, vp, vp, vp],
        "mk_set_iteration_scheme": [vp, i32],
        "mk_set_cost_model": [vp, vp],
        "mk_mlp_adam": [vp, vp, vp, vp, u32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                        ctypes.c_float, u32, vp],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.restype = i32
        f.argtypes = args
    L.mk_traversal_workspace_bytes.restype = ctypes.c_size_t
    L.mk_traversal_workspace_bytes.argtypes = [vp]
    L.mk_bfs_levels_workspace_bytes.restype = ctypes.c_size_t
    L.mk_bfs_levels_workspace_bytes.argtypes = [vp]
    L.mk_sssp_distances_workspace_bytes.restype = ctypes.c_size_t
    L.mk_sssp_distances_workspace_bytes.argtypes = [vp]
    L.mk_mlp_workspace_bytes.restype = ctypes.c_size_t
    L.mk_mlp_workspace_bytes.argtypes = [u32]
    L.mk_status_string.restype = ctypes.c_char_p
    L.mk_status_string.argtypes = [i32]
    _lib = L
    return L


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA/HIP tensors"
    return ctypes.c_void_p(t.data_ptr())


def as_u32(x, device) -> torch.Tensor:
    """Any integer tensor/array of u32 values -> contiguous int32 device tensor (bit pattern)."""
    if not torch.is_tensor(x):
        x = torch.as_tensor(x)
    if x.dtype in (torch.int64, torch.uint32):
        x = x.to(torch.int64)
        x = torch.where(x >= 2**31, x - 2**32, x).to(torch.int32)
    elif x.dtype != torch.int32:
        x = x.to(torch.int32)
    return x.to(device).contiguous()


def u32_to_i64(t: torch.Tensor) -> torch.Tensor:
    """int32 bit pattern -> the u32 value as int64."""
    return t.to(torch.int64) & 0xFFFFFFFF


def _check(st: int, what: str):
    if st != 0:
        raise MkError(st, what)


class Graph:
    """A dynamic graph resident in one arena tensor on one GPU.

    Inputs are torch integer tensors (or arrays) of u32 ids; outputs are int32 device
    tensors holding u32 bit patterns (use ``u32_to_i64`` to read them as values).
    """

    def __init__(self, n: int, src, dst, w=None, views=VIEW_FWD | VIEW_REV | VIEW_UND,
                 load_factor: float = 0.7, hash_seed: int = 1, pool_slabs: int = 0,
                 log_capacity: int = 0, device="cuda", stream: Optional[torch.cuda.Stream] = None,
                 sssp_delta: int = 0):
        self.lib = load()
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream or torch.cuda.current_stream(self.device)
        self.n = int(n)
        self.views = views | VIEW_FWD
        src = as_u32(src, self.device)
        dst = as_u32(dst, self.device)
        w = None if w is None else as_u32(w, self.device)
        m = int(src.numel())
        self.cfg = MkConfig(self.n, self.views, float(load_factor), int(hash_seed), int(pool_slabs),
                            int(log_capacity), int(sssp_delta), 0)
        nbytes = self.lib.mk_arena_bytes(ctypes.byref(self.cfg), m)
        if nbytes == 0:
            raise MkError(1, "mk_arena_bytes")
        self.arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.arena.data_ptr()) % 256
        self._arena_ptr = self.arena.data_ptr() + off
        h = ctypes.c_void_p()
        st = self.lib.mk_graph_create(ctypes.byref(self.cfg), ctypes.c_void_p(self._arena_ptr), nbytes,
                                      _ptr(src), _ptr(dst), _ptr(w), m, self._s(), ctypes.byref(h))
        _check(st, "mk_graph_create")
        self.h = h
        self.arena_bytes = nbytes

    def _s(self, stream=None):
        return ctypes.c_void_p((stream or self.stream).cuda_stream)

    def close(self):
        if getattr(self, "h", None):
            self.lib.mk_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ updates / queries
    def insert_edges(self, src, dst, w=None, status: bool = True, stream=None):
        s, d = as_u32(src, self.device), as_u32(dst, self.device)
        ww = None if w is None else as_u32(w, self.device)
        out = torch.empty(s.numel(), dtype=torch.uint8, device=self.device) if status else None
        _check(self.lib.mk_insert_edges(self.h, _ptr(s), _ptr(d), _ptr(ww), s.numel(), _ptr(out),
                                        self._s(stream)), "mk_insert_edges")
        return out

    def delete_edges(self, src, dst, status: bool = True, stream=None):
        s, d = as_u32(src, self.device), as_u32(dst, self.device)
        out = torch.empty(s.numel(), dtype=torch.uint8, device=self.device) if status else None
        _check(self.lib.mk_delete_edges(self.h, _ptr(s), _ptr(d), s.numel(), _ptr(out),
                                        self._s(stream)), "mk_delete_edges")
        return out

    def query_edges(self, src, dst, weights: bool = True, stream=None, out=None):
        """Membership (and weights) of arcs; `out` = (found u8, weight i32) preallocated."""
        s, d = as_u32(src, self.device), as_u32(dst, self.device)
        if out is None:
            found = torch.empty(s.numel(), dtype=torch.uint8, device=self.device)
            w = torch.empty(s.numel(), dtype=torch.int32, device=self.device) if weights else None
        else:
            found, w = out
        _check(self.lib.mk_query_edges(self.h, _ptr(s), _ptr(d), s.numel(), _ptr(found), _ptr(w),
                                       self._s(stream)), "mk_query_edges")
        return found, w

    def traversal_workspace(self) -> torch.Tensor:
        return torch.empty(self.lib.mk_traversal_workspace_bytes(self.h), dtype=torch.uint8,
                           device=self.device)

    def traverse_from(self, source: int, weighted: bool, ws: torch.Tensor, slot: int = 0,
                      stream=None, parents: bool = True):
        """One-off BFS (weighted=False) or SSSP from `source` in the workspace `ws`; leaves
        the graph untouched, so it may overlap other reads on other streams."""
        di = torch.empty(self.n, dtype=torch.int32, device=self.device)
        pa = torch.empty(self.n, dtype=torch.int32, device=self.device) if parents else None
        _check(self.lib.mk_traverse_from(self.h, int(source), int(bool(weighted)), _ptr(ws), ws.numel(),
                                         int(slot), _ptr(di), _ptr(pa), self._s(stream)),
               "mk_traverse_from")
        return di, pa

    def bfs_levels(self, source: int, top_down_only: bool = False, ws: Optional[torch.Tensor] = None,
                   slot: int = 0, stream=None):
        """Distance-only, direction-optimizing BFS levels (read-only on the graph).
        Returns (levels int32 tensor, number of bottom-up steps)."""
        if ws is None:
            ws = torch.empty(self.lib.mk_bfs_levels_workspace_bytes(self.h), dtype=torch.uint8,
                             device=self.device)
        lv = torch.empty(self.n, dtype=torch.int32, device=self.device)
        bu = ctypes.c_uint32()
        _check(self.lib.mk_bfs_levels(self.h, int(source), 1 if top_down_only else 0, _ptr(ws), ws.numel(),
                                      int(slot), _ptr(lv), ctypes.byref(bu), self._s(stream)),
               "mk_bfs_levels")
        return lv, int(bu.value)

    def sssp_distances(self, source: int, ws: Optional[torch.Tensor] = None, slot: int = 0, stream=None):
        """Distance-only SSSP (32-bit distances, no parents; read-only on the graph)."""
        if ws is None:
            ws = torch.empty(self.lib.mk_sssp_distances_workspace_bytes(self.h), dtype=torch.uint8,
                             device=self.device)
        di = torch.empty(self.n, dtype=torch.int32, device=self.device)
        _check(self.lib.mk_sssp_distances(self.h, int(source), _ptr(ws), ws.numel(), int(slot), _ptr(di),
                                          self._s(stream)), "mk_sssp_distances")
        return di

    # ------------------------------------------------------------ algorithms
    def bfs(self, source: int, mode: int = AUTO, parents: bool = True, stream=None):
        lv = torch.empty(self.n, dtype=torch.int32, device=self.device)
        pa = torch.empty(self.n, dtype=torch.int32, device=self.device) if parents else None
        _check(self.lib.mk_incr_bfs(self.h, int(source), _ptr(lv), _ptr(pa), mode, self._s(stream)),
               "mk_incr_bfs")
        return lv, pa

    def sssp(self, source: int, mode: int = AUTO, parents: bool = True, stream=None):
        di = torch.empty(self.n, dtype=torch.int32, device=self.device)
        pa = torch.empty(self.n, dtype=torch.int32, device=self.device) if parents else None
        _check(self.lib.mk_incr_sssp(self.h, int(source), _ptr(di), _ptr(pa), mode, self._s(stream)),
               "mk_incr_sssp")
        return di, pa

    def wcc(self, mode: int = AUTO, scheme: Optional[int] = None, stream=None):
        """Component labels (smallest id); `scheme` picks the incremental-WCC scheme
        (WCC_LOG, WCC_NAIVE, WCC_SLAB, WCC_UPDATE), None = mk_incr_wcc's default."""
        lab = torch.empty(self.n, dtype=torch.int32, device=self.device)
        if scheme is None:
            _check(self.lib.mk_incr_wcc(self.h, _ptr(lab), mode, self._s(stream)), "mk_incr_wcc")
        else:
            _check(self.lib.mk_incr_wcc_scheme(self.h, _ptr(lab), mode, int(scheme), self._s(stream)),
                   "mk_incr_wcc_scheme")
        return lab

    def set_cost_model(self, params: Optional[torch.Tensor]):
        """MLP parameters (MK_MLP_PARAMS float32 on this device) that MK_AUTO consults to pick
        incremental or recompute; None clears.  The tensor is kept alive here."""
        if params is not None:
            params = params.to(self.device, torch.float32).contiguous()
            assert params.numel() == 5187
        _check(self.lib.mk_set_cost_model(self.h, _ptr(params)), "mk_set_cost_model")
        self._cm_params = params

    def set_iteration_scheme(self, scheme: int):
        """ITER_SCHEME1 (a worker per vertex), ITER_SCHEME2 (a group per bucket chain) or
        ITER_PACKED (the default: SCHEME1, with PageRank's later iterations of a call reading
        packed in-arc keys) for the PageRank pull and the all-arc WCC walk."""
        _check(self.lib.mk_set_iteration_scheme(self.h, int(scheme)), "mk_set_iteration_scheme")

    def pagerank(self, damping: float = 0.85, tol: float = 1e-7, max_iter: int = 500,
                 mode: int = AUTO, stream=None):
        """PageRank; the default stop (iteration L1 change <= 1e-7) bounds the distance to the
        fixed point by d/(1-d) * 1e-7 = 5.7e-7 in L1, inside the 1e-6 budget with room for the
        FP32 rounding of the ranks (about 6e-8 in L1 at 4M vertices)."""
        r = torch.empty(self.n, dtype=torch.float32, device=self.device)
        it = torch.zeros(1, dtype=torch.int32, device=self.device)
        _check(self.lib.mk_incr_pagerank(self.h, float(damping), float(tol), int(max_iter), _ptr(r),
                                         _ptr(it), mode, self._s(stream)), "mk_incr_pagerank")
        return r, it

    def triangles(self, mode: int = AUTO, stream=None):
        c = torch.zeros(1, dtype=torch.int64, device=self.device)
        _check(self.lib.mk_count_triangles(self.h, _ptr(c), mode, self._s(stream)), "mk_count_triangles")
        return c

    # ------------------------------------------------------------ inspection
    def export(self):
        st = self.stats()
        cap = max(1, st["n_arcs"])
        s = torch.empty(cap, dtype=torch.int32, device=self.device)
        d = torch.empty(cap, dtype=torch.int32, device=self.device)
        w = torch.empty(cap, dtype=torch.int32, device=self.device)
        cnt = ctypes.c_uint64()
        _check(self.lib.mk_graph_export(self.h, _ptr(s), _ptr(d), _ptr(w), cap, ctypes.byref(cnt),
                                        self._s()), "mk_graph_export")
        k = int(cnt.value)
        return s[:k], d[:k], w[:k]

    def compact(self, min_tombstones: int = 1, stream=None) -> int:
        """Reclaim slabs: pack chains with tombstones, return unneeded slabs to the free
        lists.  Returns the number of slabs freed.  Must not overlap other calls."""
        out = ctypes.c_uint64()
        _check(self.lib.mk_compact(self.h, int(min_tombstones), ctypes.byref(out), self._s(stream)),
               "mk_compact")
        return int(out.value)

    def stats(self):
        out = MkStats()
        _check(self.lib.mk_graph_stats(self.h, ctypes.byref(out), self._s()), "mk_graph_stats")
        return out.as_dict()

    def probe_cost(self, op: int, view: int, src, dst) -> int:
        """Slabs the batched op would walk in one view (byte model; no change is made)."""
        s, d = as_u32(src, self.device), as_u32(dst, self.device)
        out = ctypes.c_uint64()
        _check(self.lib.mk_probe_cost(self.h, int(op), int(view), _ptr(s), _ptr(d), s.numel(),
                                      ctypes.byref(out), self._s()), "mk_probe_cost")
        return int(out.value)

    def batch_features(self, algo: int, ins=None, dels=None):
        """Cost-model features (MK_MLP_IN floats) of a batch about to be applied."""
        import numpy as np
        out = (ctypes.c_float * 12)()
        if ins is not None and ins[0].numel():
            s, d = as_u32(ins[0], self.device), as_u32(ins[1], self.device)
            w = None if len(ins) < 3 or ins[2] is None else as_u32(ins[2], self.device)
            ni = s.numel()
        else:
            s = d = w = None
            ni = 0
        if dels is not None and dels[0].numel():
            ds, dd = as_u32(dels[0], self.device), as_u32(dels[1], self.device)
            nd = ds.numel()
        else:
            ds = dd = None
            nd = 0
        _check(self.lib.mk_batch_features(self.h, int(algo), _ptr(s), _ptr(d), _ptr(w), ni, _ptr(ds),
                                          _ptr(dd), nd, out, self._s()), "mk_batch_features")
        return np.array(out[:], dtype=np.float32)

    def check(self) -> int:
        bad = ctypes.c_uint64()
        _check(self.lib.mk_graph_check(self.h, ctypes.byref(bad), self._s()), "mk_graph_check")
        return int(bad.value)
