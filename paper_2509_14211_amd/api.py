"""Convenience layer over the C ABI: a context manager that hands torch's
stream and caching allocator to the library, graph construction from R-MAT
or host edge lists, and tensor <-> vector copies.  Only marshalling: all
graph construction and PageRank arithmetic runs in libnbgrb.so.
"""
from __future__ import annotations

import numpy as np
import torch

from . import grb

RMAT_THRESHOLDS = (0.57, 0.76, 0.95)  # cumulative a, a+b, a+b+c for a=.57 b=.19 c=.19


def _torch_alloc(nbytes: int) -> int:
    return torch.cuda.caching_allocator_alloc(nbytes, stream=torch.cuda.current_stream())


def _torch_free(ptr: int) -> None:
    torch.cuda.caching_allocator_delete(ptr)


class Context:
    """GrB_init / GrB_finalize around a block, on torch's current stream."""

    def __init__(self, mode: int = grb.GrB_NONBLOCKING, torch_allocator: bool = True):
        self.mode = mode
        self.torch_allocator = torch_allocator

    def __enter__(self):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the nonblocking GraphBLAS library needs a HIP device")
        grb.GrB_init(self.mode)
        grb.GrM_set_stream(torch.cuda.current_stream().cuda_stream)
        if self.torch_allocator:
            grb.GrM_set_allocator(_torch_alloc, _torch_free)
        return self

    def __exit__(self, *exc):
        grb.GrB_finalize()
        return False


def dtype_code(dtype) -> int:
    if dtype == torch.float32:
        return grb.builtin("GrB_FP32")
    if dtype == torch.float64:
        return grb.builtin("GrB_FP64")
    if dtype == torch.int32:
        return grb.builtin("GrB_INT32")
    raise ValueError("unsupported dtype %r" % (dtype,))


class Graph:
    """CSR(A) (rows = sources), CSR(A^T) and the INT32 out-degree vector."""

    def __init__(self, n: int, A: int, AT: int, outdeg: int):
        self.n = n
        self.A = A
        self.AT = AT
        self.outdeg = outdeg
        self.m = grb.GrB_Matrix_nvals(A)

    def free(self):
        for h in (self.A, self.AT):
            if h:
                grb.GrB_Matrix_free(h)
        if self.outdeg:
            grb.GrB_Vector_free(self.outdeg)
        self.A = self.AT = self.outdeg = 0


def graph_from_device_edges(n: int, src: torch.Tensor, dst: torch.Tensor, drop_self=True) -> Graph:
    fp = grb.builtin("GrB_FP32")
    A = grb.GrB_Matrix_new(fp, n, n)
    grb.GrM_Matrix_build_edges(A, src, dst, src.numel(), drop_self)
    AT = grb.GrB_Matrix_new(fp, n, n)
    grb.GrB_transpose(AT, None, None, A, None)
    deg = grb.GrB_Vector_new(grb.builtin("GrB_INT32"), n)
    grb.GrM_Matrix_row_degree(deg, A)
    return Graph(n, A, AT, deg)


def graph_from_edges(n: int, src, dst, drop_self=True) -> Graph:
    """Graph from host (numpy uint32) edge arrays."""
    s = torch.from_numpy(np.ascontiguousarray(src, dtype=np.uint32).view(np.int32)).cuda()
    d = torch.from_numpy(np.ascontiguousarray(dst, dtype=np.uint32).view(np.int32)).cuda()
    if s.numel() == 0:
        s = torch.zeros(1, dtype=torch.int32, device="cuda")
        d = torch.zeros(1, dtype=torch.int32, device="cuda")
        g = _graph_no_edges(n)
        return g
    return graph_from_device_edges(n, s, d, drop_self)


def _graph_no_edges(n: int) -> Graph:
    fp = grb.builtin("GrB_FP32")
    A = grb.GrB_Matrix_new(fp, n, n)
    AT = grb.GrB_Matrix_new(fp, n, n)
    grb.GrB_transpose(AT, None, None, A, None)
    deg = grb.GrB_Vector_new(grb.builtin("GrB_INT32"), n)
    grb.GrM_Matrix_row_degree(deg, A)
    return Graph(n, A, AT, deg)


def rmat_device_edges(scale: int, edgefactor: int = 16, seed: int | None = None):
    m = int(edgefactor) << int(scale)
    src = torch.empty(m, dtype=torch.int32, device="cuda")
    dst = torch.empty(m, dtype=torch.int32, device="cuda")
    grb.GrM_rmat_edges(src, dst, scale, m, scale if seed is None else seed, *RMAT_THRESHOLDS)
    return src, dst


def rmat_graph(scale: int, edgefactor: int = 16, seed: int | None = None) -> Graph:
    src, dst = rmat_device_edges(scale, edgefactor, seed)
    g = graph_from_device_edges(1 << scale, src, dst, True)
    del src, dst
    return g


def web_device_edges(n: int, seed: int, model):
    """The web-shaped generator's links as device int32 tensors (the bits
    of uint32 vertex ids)."""
    m = grb.GrM_web_edges(None, None, 0, n, seed, model)
    src = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
    dst = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
    grb.GrM_web_edges(src, dst, src.numel(), n, seed, model)
    return src[:m], dst[:m]


def web_graph(n: int, seed: int, model) -> Graph:
    """Web-shaped graph (self-loops dropped, repeated links merged)."""
    src, dst = web_device_edges(n, seed, model)
    if src.numel() == 0:
        return _graph_no_edges(n)
    g = graph_from_device_edges(n, src, dst, True)
    del src, dst
    return g


def csr_of(A: int):
    """(rowptr, col) int32 tensors copied from matrix A."""
    n = grb.GrB_Matrix_nrows(A)
    nnz = grb.GrB_Matrix_nvals(A)
    rowptr = torch.empty(n + 1, dtype=torch.int32, device="cuda")
    col = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
    grb.GrM_Matrix_export_CSR(rowptr, col if nnz else None, A)
    return rowptr, col[:nnz]


def vector_from_tensor(t: torch.Tensor) -> int:
    t = t.contiguous()
    v = grb.GrB_Vector_new(dtype_code(t.dtype), t.numel())
    grb.GrM_Vector_import_dense(v, t, t.numel())
    return v


def tensor_from_vector(v: int, dtype) -> torch.Tensor:
    n = grb.GrB_Vector_size(v)
    out = torch.empty(n, dtype=dtype, device="cuda")
    grb.GrM_Vector_export_dense(out, n, v)
    return out


def pagerank(g: Graph, dtype=torch.float32, damping=0.85, tol=1e-9, itermax=1000,
             dangling=grb.GrM_DANGLING_UNIFORM, x0: torch.Tensor | None = None, check_every=8):
    """(ranks tensor, iterations, residual) from GrM_pagerank."""
    r = grb.GrB_Vector_new(dtype_code(dtype), g.n)
    xv = vector_from_tensor(x0.to(dtype)) if x0 is not None else None
    try:
        it, res = grb.GrM_pagerank(r, g.AT, g.outdeg, damping, tol, itermax, dangling, xv,
                                   check_every)
        x = tensor_from_vector(r, dtype)
    finally:
        grb.GrB_Vector_free(r)
        if xv:
            grb.GrB_Vector_free(xv)
    return x, it, res


def teleport_tensor(n: int, seeds, dtype=torch.float32) -> torch.Tensor:
    """1/|S| on the seed set S, 0 elsewhere."""
    v = torch.zeros(n, dtype=dtype, device="cuda")
    v[torch.as_tensor(list(seeds), dtype=torch.long, device="cuda")] = 1.0 / len(seeds)
    return v


def ppr(g: Graph, seeds, dtype=torch.float32, damping=0.85, tol=1e-6, itermax=1000,
        dangling=grb.GrM_DANGLING_UNIFORM, x0: int | None = None, check_every=8):
    """(ranks tensor, iterations, residual) of GrM_ppr for one seed set;
    x0 is an optional start vector handle (default: the teleport vector)."""
    tv = vector_from_tensor(teleport_tensor(g.n, seeds, dtype))
    r = grb.GrB_Vector_new(dtype_code(dtype), g.n)
    try:
        it, res = grb.GrM_ppr(r, g.AT, g.outdeg, tv, damping, tol, itermax, dangling, x0, check_every)
        x = tensor_from_vector(r, dtype)
    finally:
        grb.GrB_Vector_free(r)
        grb.GrB_Vector_free(tv)
    return x, it, res


def device_copy(ptr: int, count: int, dtype) -> torch.Tensor:
    """Copy of `count` elements of a library work buffer at device address
    ptr (the size must be a multiple of 16 bytes)."""
    out = torch.empty(count, dtype=dtype, device="cuda")
    nbytes = count * out.element_size()
    if nbytes % 16:
        raise ValueError("buffer size must be a multiple of 16 bytes")
    if nbytes:
        grb.GrM_stream_copy(out, ptr, nbytes)
    return out


def bfs_levels(g: Graph, source: int):
    """Breadth-first levels from `source` written with GraphBLAS operations
    on vectors with missing entries: the frontier's successors are
    A^T (+.second) frontier under the complement of the visited set
    (structural mask, replace), and levels<frontier> = depth.  Returns
    (levels handle (INT32, unreached vertices have no entry), depth count).
    Which operations run push (driven by the frontier's entries) or pull
    (driven by the rows of A^T), and how each vector is stored, is left to
    the library's fill estimates."""
    n = g.n
    levels = grb.GrB_Vector_new(grb.builtin("GrB_INT32"), n)
    frontier = grb.GrB_Vector_new(grb.builtin("GrB_FP32"), n)
    sem = grb.builtin("GrM_PLUS_SECOND_SEMIRING_FP32")
    second = grb.builtin("GrB_SECOND_FP32")
    try:
        grb.GrB_Vector_clear(levels)
        grb.GrB_Vector_build(frontier, [source], [1.0])
        depth = 0
        while True:
            grb.GrB_Vector_assign(levels, frontier, depth, grb.builtin("GrB_DESC_S"))
            grb.GrB_mxv(frontier, levels, None, sem, g.AT, frontier, grb.builtin("GrB_DESC_RSC"))
            # keep the frontier's values at 1 (only its pattern matters)
            grb.GrB_Vector_apply_BinaryOp2nd_FP64(frontier, None, None, second, frontier, 1.0)
            depth += 1
            if grb.GrB_Vector_nvals(frontier) == 0:
                break
    finally:
        grb.GrB_Vector_free(frontier)
    return levels, depth
