"""CPU oracle for the fused PageRank path (test infrastructure only).

This package is the reference that the HIP implementation is checked
against.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the product package never does, and this
package imports nothing from the product package.

The arithmetic lives in ``oracle.c`` (plain C, FP64, blocking mode: one
materialised pass per GraphBLAS operation of the PageRank loop in Fig. 6 of
the paper).  This module only marshals numpy arrays into it and adds the
drivers that loop over columns (personalised PageRank) or graphs.

Pins: every function here is checked by ``tests/test_oracle_*.py`` against
facts that do not come from this code -- a published SplitMix64 test vector,
brute-force set semantics for the CSR build, a dense LU solve of the
PageRank linear system, closed forms and invariants.  See the test files for
the exact list.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

DROP = 0
UNIFORM = 1

# R-MAT quadrant probabilities a, b, c, d = 0.57, 0.19, 0.19, 0.05 given as
# cumulative thresholds, written as literals so that every implementation
# compares against the same doubles.
RMAT_THRESHOLDS = (0.57, 0.76, 0.95)


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP on)."""
    if (not force and os.path.exists(_SO)
            and os.path.getmtime(_SO) >= os.path.getmtime(_SRC)):
        return _SO
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build()
        lib = ctypes.CDLL(_SO)
        i64, u64, i32, dbl = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        vp = ctypes.c_void_p
        lib.oracle_splitmix64.restype = u64
        lib.oracle_splitmix64.argtypes = [u64, u64]
        lib.oracle_rmat_edges.restype = None
        lib.oracle_rmat_edges.argtypes = [i32, i64, u64, dbl, dbl, dbl, vp, vp]
        lib.oracle_build_csr.restype = i64
        lib.oracle_build_csr.argtypes = [i64, i64, vp, vp, i32, vp, vp]
        lib.oracle_row_counts.restype = None
        lib.oracle_row_counts.argtypes = [i64, vp, vp]
        lib.oracle_transpose.restype = None
        lib.oracle_transpose.argtypes = [i64, i64, vp, vp, vp, vp]
        lib.oracle_sum.restype = dbl
        lib.oracle_sum.argtypes = [vp, i64]
        lib.oracle_pagerank.restype = i32
        lib.oracle_pagerank.argtypes = [i64, vp, vp, vp, dbl, dbl, i32, i32, i32,
                                        vp, vp, vp, vp, vp, vp]
        lib.oracle_web_degrees.restype = None
        lib.oracle_web_degrees.argtypes = [u64, u64, vp, vp]
        lib.oracle_web_edges.restype = None
        lib.oracle_web_edges.argtypes = [u64, u64, vp, vp, vp, vp]
        lib.oracle_web_row.restype = i64
        lib.oracle_web_row.argtypes = [u64, u64, vp, u64, vp]
        lib.oracle_web_links_into.restype = i64
        lib.oracle_web_links_into.argtypes = [u64, u64, vp, vp, i64, vp, vp]
        lib.oracle_set_threads.restype = None
        lib.oracle_set_threads.argtypes = [i32]
        lib.oracle_get_threads.restype = i32
        lib.oracle_get_threads.argtypes = []
        _lib = lib
        return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


# --------------------------------------------------------------------------
# Random numbers and R-MAT
# --------------------------------------------------------------------------

def splitmix64(seed: int, k: int) -> int:
    """Draw k (0-based) of the SplitMix64 stream seeded with ``seed``."""
    return int(_load().oracle_splitmix64(seed & (2**64 - 1), k & (2**64 - 1)))


def rmat_edges(scale: int, edgefactor: int, seed: int):
    """R-MAT edge list: ``edgefactor * 2**scale`` directed (src, dst) pairs
    in [0, 2**scale), before self-loop removal and deduplication."""
    m = int(edgefactor) << int(scale)
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)
    ta, tab, tabc = RMAT_THRESHOLDS
    _load().oracle_rmat_edges(int(scale), m, seed & (2**64 - 1), ta, tab, tabc,
                              _ptr(src), _ptr(dst))
    return src, dst


# --------------------------------------------------------------------------
# Web-shaped generator (stand-in for the web crawl of Section IV)
# --------------------------------------------------------------------------

WEB_FIELDS = ("kmin", "kmax", "p_zero", "p_home", "p_local", "local_min", "hub",
              "perm_a", "perm_b")


def _web_model(model) -> np.ndarray:
    return np.array([int(model[f]) for f in WEB_FIELDS], dtype=np.int64)


def web_degrees(n: int, seed: int, model) -> np.ndarray:
    """Number of generated links of every vertex (before self-loop removal
    and merging of repeats)."""
    deg = np.empty(n, dtype=np.int64)
    _load().oracle_web_degrees(int(n), seed & (2**64 - 1), _ptr(_web_model(model)), _ptr(deg))
    return deg


def web_edges(n: int, seed: int, model):
    """The generated link list (src, dst) as uint32 arrays, in order of the
    source vertex, then of the link number."""
    deg = web_degrees(n, seed, model)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=off[1:])
    m = int(off[-1])
    src = np.empty(max(m, 1), dtype=np.uint32)
    dst = np.empty(max(m, 1), dtype=np.uint32)
    _load().oracle_web_edges(int(n), seed & (2**64 - 1), _ptr(_web_model(model)), _ptr(off),
                             _ptr(src), _ptr(dst))
    return src[:m], dst[:m]


def web_graph(n: int, seed: int, model) -> "Graph":
    src, dst = web_edges(n, seed, model)
    return graph_from_edges(n, src, dst, True)


def web_row_links(n: int, seed: int, model, u: int) -> np.ndarray:
    """The generated targets of vertex u in link order (repeats and a
    self-loop included)."""
    mdl = _web_model(model)
    out = np.empty(int(mdl[1]), dtype=np.uint32)
    k = _load().oracle_web_row(int(n), seed & (2**64 - 1), _ptr(mdl), int(u), _ptr(out))
    return out[:k].copy()


def web_out_row(n: int, seed: int, model, u: int) -> np.ndarray:
    """Row u of the graph's CSR(A): distinct targets other than u, ascending."""
    t = np.unique(web_row_links(n, seed, model, u))
    return t[t != u].astype(np.int32)


def web_in_rows(n: int, seed: int, model, vertices, cap: int = 1 << 26) -> dict:
    """Rows of CSR(A^T) for the given vertices: for each v, its distinct
    in-neighbours other than v, ascending.  One scan over every link."""
    want = np.zeros(n, dtype=np.uint8)
    want[np.asarray(vertices, dtype=np.int64)] = 1
    src = np.empty(cap, dtype=np.uint32)
    dst = np.empty(cap, dtype=np.uint32)
    cnt = _load().oracle_web_links_into(int(n), seed & (2**64 - 1), _ptr(_web_model(model)),
                                        _ptr(want), int(cap), _ptr(src), _ptr(dst))
    if cnt < 0:
        raise ValueError("more than %d links into the requested vertices" % cap)
    src, dst = src[:cnt], dst[:cnt]
    rows = {}
    for v in np.unique(np.asarray(vertices, dtype=np.int64)):
        s = np.unique(src[dst == v])
        rows[int(v)] = s[s != v].astype(np.int32)
    return rows


# --------------------------------------------------------------------------
# CSR construction
# --------------------------------------------------------------------------

def build_csr(n: int, src, dst, drop_self: bool = True):
    """CSR pattern (row = source) of the edge list, duplicates merged,
    self-loops dropped when ``drop_self``.  Returns (rowptr, col) int32."""
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    rowptr = np.empty(n + 1, dtype=np.int32)
    col = np.empty(max(len(src), 1), dtype=np.int32)
    nnz = _load().oracle_build_csr(int(n), len(src), _ptr(src), _ptr(dst),
                                   1 if drop_self else 0, _ptr(rowptr), _ptr(col))
    if nnz < 0:
        raise ValueError("edge endpoint out of range")
    return rowptr, col[:nnz].copy()


def row_counts(rowptr):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    n = len(rowptr) - 1
    deg = np.empty(n, dtype=np.int32)
    _load().oracle_row_counts(n, _ptr(rowptr), _ptr(deg))
    return deg


def transpose(nrows: int, ncols: int, rowptr, col):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    rowptrT = np.empty(ncols + 1, dtype=np.int32)
    colT = np.empty(max(len(col), 1), dtype=np.int32)
    _load().oracle_transpose(int(nrows), int(ncols), _ptr(rowptr), _ptr(col),
                             _ptr(rowptrT), _ptr(colT))
    return rowptrT, colT[:len(col)].copy()


class Graph:
    """A graph as the oracle sees it: CSR(A), out-degrees, CSR(A^T)."""

    def __init__(self, n, rowptr, col):
        self.n = int(n)
        self.rowptr = rowptr
        self.col = col
        self.m = int(rowptr[-1])
        self.outdeg = row_counts(rowptr)
        self.rowptrT, self.colT = transpose(self.n, self.n, rowptr, col)
        self.indeg = row_counts(self.rowptrT)


def graph_from_edges(n, src, dst, drop_self=True) -> Graph:
    rowptr, col = build_csr(n, src, dst, drop_self)
    return Graph(n, rowptr, col)


def rmat_graph(scale: int, edgefactor: int = 16, seed: int | None = None) -> Graph:
    """R-MAT graph with self-loops dropped and duplicates merged; the seed
    defaults to the scale."""
    src, dst = rmat_edges(scale, edgefactor, scale if seed is None else seed)
    return graph_from_edges(1 << scale, src, dst, True)


# --------------------------------------------------------------------------
# PageRank
# --------------------------------------------------------------------------

class PRResult:
    def __init__(self, x, iters, resid, rho_hist, D_hist):
        self.x = x
        self.iters = iters
        self.resid = resid
        self.rho_hist = rho_hist
        self.D_hist = D_hist


def pagerank(g: Graph, damping=0.85, tol=1e-9, itermax=1000, mode=UNIFORM,
             v=None, x0=None, fixed_iters=0) -> PRResult:
    """Blocking FP64 PageRank (Fig. 6 loop, one pass per operation).

    ``v`` is the teleport distribution (None: uniform 1/n), ``x0`` the start
    vector (None: v).  ``mode`` DROP reproduces the paper's variant that does
    not redistribute dangling rank; UNIFORM returns it through v.
    ``fixed_iters`` > 0 runs exactly that many passes."""
    n = g.n
    cap = max(itermax, fixed_iters, 1)
    x = np.empty(max(n, 1), dtype=np.float64)
    rho_hist = np.zeros(cap, dtype=np.float64)
    D_hist = np.zeros(cap + 1, dtype=np.float64)
    resid = ctypes.c_double(0.0)
    vv = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
    xx = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    if vv is not None and len(vv) != n:
        raise ValueError("v has the wrong length")
    if xx is not None and len(xx) != n:
        raise ValueError("x0 has the wrong length")
    it = _load().oracle_pagerank(
        n, _ptr(g.rowptrT), _ptr(g.colT), _ptr(g.outdeg), float(damping), float(tol),
        int(itermax), int(fixed_iters), int(mode), _ptr(vv), _ptr(xx), _ptr(x),
        _ptr(rho_hist), _ptr(D_hist), ctypes.byref(resid))
    return PRResult(x[:n].copy(), int(it), float(resid.value), rho_hist[:it].copy(),
                    D_hist[:it + 1].copy())


def teleport_vector(n: int, seeds) -> np.ndarray:
    """Personalised teleport distribution: uniform over the seed set."""
    seeds = np.asarray(seeds, dtype=np.int64)
    v = np.zeros(n, dtype=np.float64)
    v[seeds] = 1.0 / len(seeds)
    return v


def ppr(g: Graph, seeds, damping=0.85, tol=1e-6, itermax=1000, fixed_iters=0,
        mode=UNIFORM, x0=None) -> PRResult:
    """Personalised PageRank of one seed set: teleport and dangling mass go
    to the seeds, start vector = teleport vector unless x0 is given."""
    v = teleport_vector(g.n, seeds)
    return pagerank(g, damping, tol, itermax, mode, v=v, x0=x0, fixed_iters=fixed_iters)


def ppr_batch(g: Graph, seed_sets, damping=0.85, tol=1e-6, itermax=1000,
              fixed_iters=0, mode=UNIFORM):
    """One single-vector solve per seed set; returns a list of PRResult."""
    return [ppr(g, s, damping, tol, itermax, fixed_iters, mode) for s in seed_sets]


def oracle_sum(x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float64)
    return float(_load().oracle_sum(_ptr(x), len(x)))
