"""CPU oracle for block-based triangle counting -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and the
two share no code.  The arithmetic lives in ``oracle.c`` (plain C + OpenMP);
this file only marshals numpy arrays.

Functions follow arXiv 2009.12457:
  * ``total``        -- Alg. 2 (TC-Intersect) over the degree-ordered,
                        oriented graph, with Alg. 1 as the list intersection.
  * ``total_rows``   -- Alg. 2 over a list of rows (bounded timing samples).
  * ``total_hmap``   -- Alg. 3 (TC-HMap), a second, independent count.
  * ``cuts``         -- the cut rule used for the p x p symmetric rectilinear
                        partition (the paper's partitioner is not described in
                        it; see the header of oracle.c for the reading).
  * ``task_list``    -- Alg. 4 (bbTaskComposition) order.
  * ``tasks``        -- per-task counts: each triangle with ranks a<b<c is
                        assigned to task (part(a), part(b), part(c)) (Sec. 4.2).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        P32, P64, PU64 = (ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64),
                          ctypes.POINTER(ctypes.c_uint64))
        L.or_build_edges.argtypes = [i64, i64, P32, P32]
        L.or_build_edges.restype = vp
        L.or_build_csr.argtypes = [i64, P64, P32]
        L.or_build_csr.restype = vp
        L.or_free.argtypes = [vp]
        L.or_n.argtypes = [vp]
        L.or_n.restype = i64
        L.or_m.argtypes = [vp]
        L.or_m.restype = i64
        L.or_rank.argtypes = [vp, P32]
        L.or_degree.argtypes = [vp, P64]
        L.or_oriented.argtypes = [vp, P64, P32]
        L.or_total.argtypes = [vp, ctypes.c_int]
        L.or_total.restype = ctypes.c_uint64
        L.or_total_rows.argtypes = [vp, P64, i64, ctypes.c_int]
        L.or_total_rows.restype = ctypes.c_uint64
        L.or_total_hmap.argtypes = [vp, ctypes.c_int]
        L.or_total_hmap.restype = ctypes.c_uint64
        L.or_cuts.argtypes = [vp, i32, ctypes.c_int, P32]
        L.or_cuts.restype = ctypes.c_int
        L.or_task_list.argtypes = [i32, P32]
        L.or_task_list.restype = i64
        L.or_tasks.argtypes = [vp, i32, P32, PU64, PU64, ctypes.c_int]
        L.or_tasks.restype = ctypes.c_uint64
        L.or_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def max_threads() -> int:
    return int(_load().or_max_threads())


CUT_BALANCED = 0
CUT_UNIFORM = 1


class OracleGraph:
    """The oracle's own canonical, degree-ordered, oriented copy of a graph."""

    def __init__(self, n, src=None, dst=None, rowptr=None, colidx=None):
        L = _load()
        self.n = int(n)
        if rowptr is not None:
            rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
            colidx = np.ascontiguousarray(colidx, dtype=np.int32)
            h = L.or_build_csr(self.n, _p(rowptr, ctypes.c_int64), _p(colidx, ctypes.c_int32))
        else:
            src = np.ascontiguousarray(src, dtype=np.int32)
            dst = np.ascontiguousarray(dst, dtype=np.int32)
            h = L.or_build_edges(self.n, len(src), _p(src, ctypes.c_int32), _p(dst, ctypes.c_int32))
        if not h:
            raise ValueError("oracle: bad graph input")
        self._h = h
        self.m = int(L.or_m(h))

    @classmethod
    def from_graph(cls, g):
        return cls(g.n, rowptr=g.rowptr, colidx=g.colidx)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().or_free(h)
            self._h = None

    def rank(self) -> np.ndarray:
        out = np.empty(self.n, np.int32)
        _load().or_rank(self._h, _p(out, ctypes.c_int32))
        return out

    def degree(self) -> np.ndarray:
        out = np.empty(self.n, np.int64)
        _load().or_degree(self._h, _p(out, ctypes.c_int64))
        return out

    def oriented(self):
        orow = np.empty(self.n + 1, np.int64)
        ocol = np.empty(self.m, np.int32)
        _load().or_oriented(self._h, _p(orow, ctypes.c_int64), _p(ocol, ctypes.c_int32))
        return orow, ocol

    def total(self, threads: int = 0) -> int:
        return int(_load().or_total(self._h, threads or max_threads()))

    def total_rows(self, rows, threads: int = 0) -> int:
        """Alg. 2 over the listed rows (ranks) only."""
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        r = int(_load().or_total_rows(self._h, _p(rows, ctypes.c_int64), len(rows), threads or max_threads()))
        if r == (1 << 64) - 1:
            raise ValueError("oracle: row out of range")
        return r

    def total_hmap(self, threads: int = 0) -> int:
        return int(_load().or_total_hmap(self._h, threads or max_threads()))

    def cuts(self, p: int, mode: int = CUT_BALANCED) -> np.ndarray:
        out = np.empty(p + 1, np.int32)
        if _load().or_cuts(self._h, p, mode, _p(out, ctypes.c_int32)) != 0:
            raise ValueError("oracle: p out of range")
        return out

    def tasks(self, p: int, cuts=None, threads: int = 0):
        """(total, per_task[|T|] in Alg. 4 order, block_nnz[p(p+1)/2])."""
        if cuts is None:
            cuts = self.cuts(p)
        cuts = np.ascontiguousarray(cuts, dtype=np.int32)
        nt = p * (p + 1) * (p + 2) // 6
        per = np.zeros(nt, np.uint64)
        bn = np.zeros(p * (p + 1) // 2, np.uint64)
        tot = _load().or_tasks(self._h, p, _p(cuts, ctypes.c_int32), _p(per, ctypes.c_uint64),
                               _p(bn, ctypes.c_uint64), threads or max_threads())
        if tot == (1 << 64) - 1:
            raise ValueError("oracle: invalid cuts")
        return int(tot), per, bn


def task_list(p: int) -> np.ndarray:
    """Alg. 4 order, shape (|T|, 3)."""
    L = _load()
    nt = int(L.or_task_list(p, None))
    out = np.empty((nt, 3), np.int32)
    L.or_task_list(p, _p(out, ctypes.c_int32))
    return out
