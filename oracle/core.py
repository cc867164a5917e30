"""ctypes front end of the C oracle (``htri_oracle.c``) -- test infrastructure only.

The shared library is compiled by :func:`build` (gcc, plain C11 + pthreads);
``__graft_entry__.build()`` calls it so that the checker exists wherever the
product library is built.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "htri_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

ORC_OK = 0
_ERRORS = {-1: "invalid", -2: "range", -3: "empty hyperedge", -4: "duplicate hyperedge",
           -5: "out of memory", -8: "state"}


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what}: {_ERRORS.get(code, code)}")
        self.code = code


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32, u32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
    lib.orc_normalize.argtypes = [P, i64, P, i32, ctypes.c_int, ctypes.POINTER(P)]
    lib.orc_normalize.restype = ctypes.c_int
    for f in ("orc_num_edges", "orc_nnz", "orc_removed", "orc_num_wedges"):
        getattr(lib, f).argtypes = [P]
        getattr(lib, f).restype = i64
    lib.orc_get_csr.argtypes = [P, P, P, P]
    lib.orc_build_wedges.argtypes = [P]
    lib.orc_build_wedges.restype = ctypes.c_int
    lib.orc_build_wedges_threads.argtypes = [P, ctypes.c_int]
    lib.orc_build_wedges_threads.restype = ctypes.c_int
    lib.orc_summary.argtypes = [P, P]
    lib.orc_get_wedges.argtypes = [P, P, P, P]
    lib.orc_get_degrees.argtypes = [P, P]
    lib.orc_count.argtypes = [P, ctypes.c_int, u32, P, P, P]
    lib.orc_count.restype = ctypes.c_int
    lib.orc_count_range.argtypes = [P, i64, i64, ctypes.c_int, u32, P, P, P]
    lib.orc_count_range.restype = ctypes.c_int
    lib.orc_wedge_closure.argtypes = [P, P, P, i64, P]
    lib.orc_wedge_closure.restype = ctypes.c_int
    lib.orc_build_vertex_lists.argtypes = [P]
    lib.orc_build_vertex_lists.restype = ctypes.c_int
    lib.orc_wedge_closure_ranked.argtypes = [P, P, P, P, i64, P]
    lib.orc_wedge_closure_ranked.restype = ctypes.c_int
    lib.orc_edge_triangles.argtypes = [P, P, i64, u32, P]
    lib.orc_edge_triangles.restype = ctypes.c_int
    lib.orc_count_owner_sample.argtypes = [P, P, i64, ctypes.c_int, P, P]
    lib.orc_count_owner_sample.restype = ctypes.c_int
    lib.orc_classify.argtypes = [i64] * 7
    lib.orc_classify.restype = ctypes.c_int
    lib.orc_free.argtypes = [P]
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def classify(si, sj, sk, wij, wik, wjk, g) -> int:
    """Pattern number of a hyper-triangle from its sizes and common-vertex counts."""
    return int(_load().orc_classify(si, sj, sk, wij, wik, wjk, g))


@dataclass
class CountResult:
    H: np.ndarray            # int64[21]; H[0] = total
    t: Optional[np.ndarray]  # int64[m] per-hyperedge counts (normalised ids)
    cw: Optional[np.ndarray] # int32[|wedges|] forward closure per wedge


class OracleGraph:
    """A normalised hypergraph held by the C oracle."""

    def __init__(self, offsets: np.ndarray, members: np.ndarray, num_vertices: int,
                 dedupe: bool = True):
        lib = _load()
        self._lib = lib
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        mem = np.ascontiguousarray(members, dtype=np.int32)
        h = ctypes.c_void_p()
        rc = lib.orc_normalize(_ptr(off), off.shape[0] - 1, _ptr(mem), int(num_vertices),
                               1 if dedupe else 0, ctypes.byref(h))
        if rc != ORC_OK:
            raise OracleError(rc, "normalize")
        self._h = h
        self.num_vertices = int(num_vertices)
        self.m = int(lib.orc_num_edges(h))
        self.removed = int(lib.orc_removed(h))
        self._wedges_built = False

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.orc_free(h)
            self._h = None

    # -- normalised CSR -------------------------------------------------
    def csr(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        nnz = int(self._lib.orc_nnz(self._h))
        off = np.empty(self.m + 1, np.int64)
        mem = np.empty(nnz, np.int32)
        orig = np.empty(self.m, np.int64)
        self._lib.orc_get_csr(self._h, _ptr(off), _ptr(mem), _ptr(orig))
        return off, mem, orig

    # -- step 1 ---------------------------------------------------------
    def build_wedges(self, nthreads: int = 1) -> None:
        """Step 1; owners are split over nthreads threads (same result for
        any count)."""
        if not self._wedges_built:
            rc = self._lib.orc_build_wedges_threads(self._h, int(max(1, nthreads)))
            if rc != ORC_OK:
                raise OracleError(rc, "build_wedges")
            self._wedges_built = True

    def summary(self) -> np.ndarray:
        """[|wedges|, |intersection|, |inclusion|, W, max omega, m]"""
        self.build_wedges()
        out = np.zeros(6, np.int64)
        self._lib.orc_summary(self._h, _ptr(out))
        return out

    def wedges(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        self.build_wedges()
        nw = int(self._lib.orc_num_wedges(self._h))
        wi = np.empty(nw, np.int32)
        wj = np.empty(nw, np.int32)
        wo = np.empty(nw, np.int32)
        self._lib.orc_get_wedges(self._h, _ptr(wi), _ptr(wj), _ptr(wo))
        return wi, wj, wo

    def degrees(self) -> np.ndarray:
        self.build_wedges()
        d = np.empty(self.m, np.int64)
        self._lib.orc_get_degrees(self._h, _ptr(d))
        return d

    # -- step 2 ---------------------------------------------------------
    def count(self, nthreads: int = 0, edge_mask: int = 0x1FFFFE, per_edge: bool = True,
              per_wedge: bool = False) -> CountResult:
        self.build_wedges()
        if nthreads <= 0:
            nthreads = max(1, min(16, os.cpu_count() or 1))
        H = np.zeros(21, np.int64)
        t = np.zeros(self.m, np.int64) if per_edge else None
        cw = np.zeros(int(self._lib.orc_num_wedges(self._h)), np.int32) if per_wedge else None
        rc = self._lib.orc_count(self._h, int(nthreads), ctypes.c_uint32(edge_mask), _ptr(H),
                                 _ptr(t), _ptr(cw))
        if rc != ORC_OK:
            raise OracleError(rc, "count")
        return CountResult(H, t, cw)

    def count_range(self, i0: int, i1: int, nthreads: int = 0, edge_mask: int = 0x1FFFFE,
                    per_edge: bool = True) -> CountResult:
        """The count restricted to owners [i0, i1) (triangles whose smallest
        id lies there); results over ranges tiling [0, m) sum to count()."""
        self.build_wedges()
        if nthreads <= 0:
            nthreads = max(1, min(16, os.cpu_count() or 1))
        H = np.zeros(21, np.int64)
        t = np.zeros(self.m, np.int64) if per_edge else None
        rc = self._lib.orc_count_range(self._h, int(i0), int(i1), int(nthreads),
                                       ctypes.c_uint32(edge_mask), _ptr(H), _ptr(t), None)
        if rc != ORC_OK:
            raise OracleError(rc, "count_range")
        return CountResult(H, t, None)

    def wedge_closure(self, wi: np.ndarray, wj: np.ndarray) -> np.ndarray:
        """int64[n, 21] per-pattern forward closure of the given wedges (i<j)."""
        self.build_wedges()
        wi = np.ascontiguousarray(wi, dtype=np.int32)
        wj = np.ascontiguousarray(wj, dtype=np.int32)
        out = np.zeros((wi.shape[0], 21), np.int64)
        rc = self._lib.orc_wedge_closure(self._h, _ptr(wi), _ptr(wj), wi.shape[0], _ptr(out))
        if rc != ORC_OK:
            raise OracleError(rc, "wedge_closure")
        return out


    def wedge_closure_ranked(self, rank: Optional[np.ndarray], wi: np.ndarray,
                             wj: np.ndarray) -> np.ndarray:
        """int64[n, 21]: closure of wedges (i, j), rank[i] < rank[j], by the
        third hyperedges k with rank[k] > rank[j] (rank None = id order).
        Needs only the vertex lists, so it scales to graphs where
        build_wedges/count would be too slow."""
        wi = np.ascontiguousarray(wi, dtype=np.int32)
        wj = np.ascontiguousarray(wj, dtype=np.int32)
        rk = None if rank is None else np.ascontiguousarray(rank, dtype=np.int64)
        out = np.zeros((wi.shape[0], 21), np.int64)
        rc = self._lib.orc_wedge_closure_ranked(self._h, _ptr(rk), _ptr(wi), _ptr(wj), wi.shape[0],
                                                _ptr(out))
        if rc != ORC_OK:
            raise OracleError(rc, "wedge_closure_ranked")
        return out

    def edge_triangles(self, xs: np.ndarray, edge_mask: int = 0x1FFFFE) -> np.ndarray:
        """Per listed hyperedge: triangles containing it (patterns in edge_mask)."""
        xs = np.ascontiguousarray(xs, dtype=np.int32)
        out = np.zeros(xs.shape[0], np.int64)
        rc = self._lib.orc_edge_triangles(self._h, _ptr(xs), xs.shape[0], ctypes.c_uint32(edge_mask),
                                          _ptr(out))
        if rc != ORC_OK:
            raise OracleError(rc, "edge_triangles")
        return out

    def count_owner_sample(self, owners: np.ndarray, nthreads: int = 0):
        """(H int64[21], hyperwedges closed) over the listed owners only."""
        owners = np.ascontiguousarray(owners, dtype=np.int32)
        if nthreads <= 0:
            nthreads = max(1, min(16, os.cpu_count() or 1))
        H = np.zeros(21, np.int64)
        nw = ctypes.c_int64(0)
        rc = self._lib.orc_count_owner_sample(self._h, _ptr(owners), owners.shape[0], int(nthreads),
                                              _ptr(H), ctypes.byref(nw))
        if rc != ORC_OK:
            raise OracleError(rc, "count_owner_sample")
        return H, int(nw.value)


def prec_rank(offsets: np.ndarray, members: np.ndarray, num_vertices: int) -> np.ndarray:
    """rank[x] of normalised hyperedge x in the order (delta_x, x) ascending,
    delta_x = sum over v in e_x of (|E_v| - 1)."""
    m = offsets.shape[0] - 1
    dv = np.bincount(members, minlength=num_vertices).astype(np.int64)
    owner = np.repeat(np.arange(m, dtype=np.int64), np.diff(offsets))
    delta = np.zeros(m, np.int64)
    np.add.at(delta, owner, dv[members] - 1)
    order = np.lexsort((np.arange(m), delta))
    rank = np.empty(m, np.int64)
    rank[order] = np.arange(m)
    return rank


def permuted(offsets: np.ndarray, members: np.ndarray, order: np.ndarray):
    """Relabel hyperedges: new id r holds old hyperedge order[r]."""
    sizes = np.diff(offsets)[order]
    off = np.zeros(order.shape[0] + 1, np.int64)
    np.cumsum(sizes, out=off[1:])
    idx = np.concatenate([np.arange(offsets[x], offsets[x + 1]) for x in order]) if order.size else np.zeros(0, np.int64)
    return off, members[idx].astype(np.int32)
