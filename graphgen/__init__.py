"""Seeded synthetic graphs: R-MAT, Erdos-Renyi G(n,p) and simple-graph CSR.

This module is the one input source shared by the GPU library's tests and
benchmarks and by the CPU oracle.  It holds no triangle-counting arithmetic:
it draws edges (counter-based SplitMix64, so results do not depend on the
thread count) and canonicalises an edge multiset into a simple undirected
graph stored as a symmetric CSR with sorted rows, no self-loops and no
duplicate entries.  The C code is in ``graphgen.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgraphgen.so")
_SRC = os.path.join(_HERE, "graphgen.c")

# Default R-MAT quadrant probabilities (a, b, c); d = 1 - a - b - c = 0.05.
RMAT_ABC = (0.57, 0.19, 0.19)


def build(force: bool = True) -> str:
    """Compiles libgraphgen.so with gcc/OpenMP and returns its path."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        lib = ctypes.CDLL(_SO)
        i64, i32p, i64p, f64, u64 = (ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.c_double, ctypes.c_uint64)
        lib.gg_rmat_edges.argtypes = [ctypes.c_int, i64, f64, f64, f64, u64, i32p, i32p]
        lib.gg_rmat_edges.restype = ctypes.c_int
        lib.gg_er_count.argtypes = [i64, f64, u64]
        lib.gg_er_count.restype = i64
        lib.gg_er_edges.argtypes = [i64, f64, u64, i64, i32p, i32p]
        lib.gg_er_edges.restype = ctypes.c_int
        lib.gg_csr_from_edges.argtypes = [i64, i64, i32p, i32p, i64p, i32p, i64]
        lib.gg_csr_from_edges.restype = i64
        lib.gg_rmat_csr.argtypes = [ctypes.c_int, i64, f64, f64, f64, u64, i64p, i32p, i64]
        lib.gg_rmat_csr.restype = i64
        lib.gg_er_csr.argtypes = [i64, f64, u64, i64p, i32p, i64]
        lib.gg_er_csr.restype = i64
        _lib = lib
    return _lib


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _p64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


@dataclass
class Graph:
    """Simple undirected graph as a symmetric CSR (both directions stored)."""

    n: int
    rowptr: np.ndarray  # int64[n+1]
    colidx: np.ndarray  # int32[2m], rows strictly increasing
    name: str = ""

    @property
    def m(self) -> int:
        """Undirected edge count."""
        return int(self.rowptr[-1]) // 2

    def edges(self):
        """Each undirected edge once, as (u, v) with u < v."""
        src = np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.rowptr))
        keep = src < self.colidx
        return src[keep], self.colidx[keep]


def rmat_edges(scale: int, edge_factor: int, seed: int, abc=RMAT_ABC):
    """Raw R-MAT samples (duplicates and self-loops kept): 2^scale * edge_factor pairs."""
    ne = (1 << scale) * edge_factor
    src = np.empty(ne, np.int32)
    dst = np.empty(ne, np.int32)
    rc = _load().gg_rmat_edges(scale, ne, abc[0], abc[1], abc[2], seed, _p32(src), _p32(dst))
    if rc != 0:
        raise ValueError(f"gg_rmat_edges failed ({rc})")
    return src, dst


def er_edges(n: int, p: float, seed: int):
    """Raw G(n,p) pairs (v, w) with w < v."""
    lib = _load()
    ne = lib.gg_er_count(n, p, seed)
    src = np.empty(ne, np.int32)
    dst = np.empty(ne, np.int32)
    rc = lib.gg_er_edges(n, p, seed, ne, _p32(src), _p32(dst))
    if rc != 0:
        raise ValueError(f"gg_er_edges failed ({rc})")
    return src, dst


def _finish(n, rowptr, col, kept, name):
    if kept < 0:
        raise ValueError(f"graph construction failed ({kept})")
    return Graph(n=n, rowptr=rowptr, colidx=col[:kept], name=name)


def from_edges(n: int, src, dst, name: str = "") -> Graph:
    """Canonical simple graph from any edge multiset (loops and repeats dropped)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    rowptr = np.empty(n + 1, np.int64)
    cap = max(2 * len(src), 1)
    col = np.empty(cap, np.int32)
    kept = _load().gg_csr_from_edges(n, len(src), _p32(src), _p32(dst), _p64(rowptr), _p32(col), cap)
    return _finish(n, rowptr, col, kept, name)


def rmat(scale: int, edge_factor: int, seed: int, abc=RMAT_ABC) -> Graph:
    """R-MAT graph on 2^scale ids from 2^scale * edge_factor samples, canonicalised."""
    n = 1 << scale
    ne = n * edge_factor
    rowptr = np.empty(n + 1, np.int64)
    cap = max(2 * ne, 1)
    col = np.empty(cap, np.int32)
    kept = _load().gg_rmat_csr(scale, ne, abc[0], abc[1], abc[2], seed, _p64(rowptr), _p32(col), cap)
    return _finish(n, rowptr, col, kept, f"rmat-s{scale}-ef{edge_factor}-seed{seed}")


def er(n: int, p: float, seed: int) -> Graph:
    """Erdos-Renyi G(n, p) graph."""
    lib = _load()
    ne = lib.gg_er_count(n, p, seed)
    rowptr = np.empty(n + 1, np.int64)
    cap = max(2 * ne, 1)
    col = np.empty(cap, np.int32)
    kept = lib.gg_er_csr(n, p, seed, _p64(rowptr), _p32(col), cap)
    return _finish(n, rowptr, col, kept, f"er-n{n}-p{p:.6g}-seed{seed}")


def er_avgdeg(n: int, avg_degree: float, seed: int) -> Graph:
    """G(n, p) with p = avg_degree / (n - 1)."""
    return er(n, float(avg_degree) / float(max(n - 1, 1)), seed)


def relabel(g: Graph, seed: int) -> Graph:
    """The same graph under a seeded random permutation of vertex ids."""
    rng = np.random.default_rng(seed)
    pi = rng.permutation(g.n).astype(np.int32)
    u, v = g.edges()
    return from_edges(g.n, pi[u], pi[v], name=g.name + f"-relabel{seed}")


# Named workloads (sizes and seeds of the benchmark configurations).
def workload(name: str) -> Graph:
    if name == "er2000":
        return er(2000, 0.005, 1)
    if name == "rmat20":
        return rmat(20, 16, 20)
    if name == "rmat24":
        return rmat(24, 16, 24)
    if name == "er24":
        return er_avgdeg(1 << 24, 32.0, 2)
    if name == "rmat27":
        return rmat(27, 16, 27)
    if name.startswith("rmat"):  # rmatS[_efE]
        body = name[4:]
        ef = 16
        if "_ef" in body:
            body, e = body.split("_ef")
            ef = int(e)
        s = int(body)
        return rmat(s, ef, s)
    raise KeyError(name)
