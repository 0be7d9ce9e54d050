"""Python binding of libnbgrb.so (include/nbgrb.h).

The functions keep the C names and argument order; output handles that C
returns through a pointer are returned instead, and GrB_Info codes other
than success (and GrB_NO_VALUE where documented) raise GrBError.  Device
buffers are passed as torch tensors on the current CUDA (HIP) device or as
raw integer addresses.  No arithmetic happens here: every step runs in the
library's kernels.  The library must be built; nothing falls back to
another implementation when it is not.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnbgrb.so")

GrB_SUCCESS = 0
GrB_NO_VALUE = 1
GrB_NONBLOCKING = 0
GrB_BLOCKING = 1
GrB_COMPLETE = 0
GrB_MATERIALIZE = 1
GrM_DANGLING_DROP = 0
GrM_DANGLING_UNIFORM = 1

_INFO_NAMES = {
    0: "GrB_SUCCESS", 1: "GrB_NO_VALUE", -1: "GrB_UNINITIALIZED_OBJECT", -2: "GrB_NULL_POINTER",
    -3: "GrB_INVALID_VALUE", -4: "GrB_INVALID_INDEX", -5: "GrB_DOMAIN_MISMATCH",
    -6: "GrB_DIMENSION_MISMATCH", -7: "GrB_OUTPUT_NOT_EMPTY", -8: "GrB_NOT_IMPLEMENTED",
    -101: "GrB_PANIC", -102: "GrB_OUT_OF_MEMORY", -103: "GrB_INSUFFICIENT_SPACE",
    -104: "GrB_INVALID_OBJECT", -105: "GrB_INDEX_OUT_OF_BOUNDS", -106: "GrB_EMPTY_OBJECT",
}

# The info codes as module constants (GrB_INVALID_VALUE, ...).
globals().update({name: code for code, name in _INFO_NAMES.items()})

# Data symbols exported by the library (types, operators, descriptors).
DATA_SYMBOLS = [
    "GrB_BOOL", "GrB_INT32", "GrB_FP32", "GrB_FP64",
    "GrB_IDENTITY_FP32", "GrB_IDENTITY_FP64", "GrB_ABS_FP32", "GrB_ABS_FP64",
    "GrB_AINV_FP32", "GrB_AINV_FP64", "GrB_MINV_FP32", "GrB_MINV_FP64",
    "GrM_MINV_OR_ZERO_FP32", "GrM_MINV_OR_ZERO_FP64",
    "GrB_PLUS_FP32", "GrB_PLUS_FP64", "GrB_MINUS_FP32", "GrB_MINUS_FP64",
    "GrB_TIMES_FP32", "GrB_TIMES_FP64", "GrB_DIV_FP32", "GrB_DIV_FP64",
    "GrB_MAX_FP32", "GrB_MAX_FP64", "GrB_MIN_FP32", "GrB_MIN_FP64",
    "GrB_FIRST_FP32", "GrB_FIRST_FP64", "GrB_SECOND_FP32", "GrB_SECOND_FP64",
    "GrM_ABSDIFF_FP32", "GrM_ABSDIFF_FP64",
    "GrB_PLUS_MONOID_FP32", "GrB_PLUS_MONOID_FP64",
    "GrB_PLUS_TIMES_SEMIRING_FP32", "GrB_PLUS_TIMES_SEMIRING_FP64",
    "GrM_PLUS_SECOND_SEMIRING_FP32", "GrM_PLUS_SECOND_SEMIRING_FP64",
    "GrB_DESC_C", "GrB_DESC_S", "GrB_DESC_SC", "GrB_DESC_R", "GrB_DESC_RC", "GrB_DESC_RS", "GrB_DESC_RSC",
    "GrM_BF16",
]

vp = ctypes.c_void_p
u64 = ctypes.c_uint64
i64 = ctypes.c_int64
i32 = ctypes.c_int
dbl = ctypes.c_double
PV = ctypes.POINTER(ctypes.c_void_p)


class GrM_PlanConfig(ctypes.Structure):
    _fields_ = [("kernel", i32), ("lds_entries", i32), ("lds_rows", i32), ("long_row", i32),
                ("chunk", i32), ("grid", i32), ("hot", i32), ("relabel", i32), ("xcd_split", i32)]


class GrM_WebModel(ctypes.Structure):
    _fields_ = [("kmin", i32), ("kmax", i32), ("p_zero", i32), ("p_home", i32), ("p_local", i32),
                ("local_min", i32), ("hub", i32), ("perm_a", ctypes.c_uint32), ("perm_b", ctypes.c_uint32)]


class GrM_Stats(ctypes.Structure):
    _fields_ = [("kernels", i64), ("fused_launches", i64), ("plan_hits", i64),
                ("plan_misses", i64), ("elided_nodes", i64), ("forced_waits", i64),
                ("ewise_fused", i64), ("ewise_ops", i64), ("jit_compiles", i64),
                ("jit_disk_hits", i64), ("jit_memory_hits", i64), ("mxv_push", i64), ("mxv_pull", i64),
                ("out_full", i64), ("out_bitset", i64), ("out_sparse", i64), ("index_loops", i64),
                ("range_loops", i64), ("device_allocs", i64)]


# name -> (restype, argtypes).  All return GrB_Info unless noted.
_FUNCS = {
    "GrB_init": [i32],
    "GrB_finalize": [],
    "GrM_get_mode": [ctypes.POINTER(i32)],
    "GrM_set_mode": [i32],
    "GrM_set_stream": [vp],
    "GrM_set_allocator": [vp, vp, vp],
    "GrM_fail_allocation_after": [i64],
    "GrM_get_stats": [ctypes.POINTER(GrM_Stats)],
    "GrM_reset_stats": [],
    "GrM_set_fusion": [i32],
    "GrB_Vector_nvals": [ctypes.POINTER(u64), vp],
    "GrB_Vector_clear": [vp],
    "GrB_Vector_build_FP32": [vp, vp, vp, u64, vp],
    "GrB_Vector_build_FP64": [vp, vp, vp, u64, vp],
    "GrB_Vector_build_INT32": [vp, vp, vp, u64, vp],
    "GrB_Vector_extractTuples_FP32": [vp, vp, ctypes.POINTER(u64), vp],
    "GrB_Vector_extractTuples_FP64": [vp, vp, ctypes.POINTER(u64), vp],
    "GrB_Vector_extractTuples_INT32": [vp, vp, ctypes.POINTER(u64), vp],
    "GrB_Vector_assign_FP32": [vp, vp, vp, ctypes.c_float, vp, u64, vp],
    "GrB_Vector_assign_FP64": [vp, vp, vp, dbl, vp, u64, vp],
    "GrB_Vector_assign_INT32": [vp, vp, vp, i32, vp, u64, vp],
    "GrM_Vector_format": [ctypes.POINTER(i32), vp],
    "GrM_set_format_policy": [i32],
    "GrM_set_many_team_max": [i32],
    "GrM_set_many_team_wait": [ctypes.c_ulonglong],
    "GrM_code_cache_clear": [],
    "GrB_Scalar_new": [PV, vp],
    "GrB_Scalar_free": [PV],
    "GrB_Scalar_setElement_FP64": [vp, dbl],
    "GrB_Scalar_extractElement_FP64": [ctypes.POINTER(dbl), vp],
    "GrB_Scalar_wait": [vp, i32],
    "GrM_Scalar_affine": [vp, dbl, vp, dbl],
    "GrB_Vector_new": [PV, vp, u64],
    "GrB_Vector_free": [PV],
    "GrB_Vector_dup": [PV, vp],
    "GrB_Vector_size": [ctypes.POINTER(u64), vp],
    "GrM_Vector_type": [PV, vp],
    "GrB_Vector_wait": [vp, i32],
    "GrM_Vector_fill": [vp, dbl],
    "GrM_Vector_import_dense": [vp, vp, u64],
    "GrM_Vector_export_dense": [vp, u64, vp],
    "GrM_Vector_device_pointer": [PV, vp],
    "GrB_Matrix_new": [PV, vp, u64, u64],
    "GrB_Matrix_free": [PV],
    "GrB_Matrix_nrows": [ctypes.POINTER(u64), vp],
    "GrB_Matrix_ncols": [ctypes.POINTER(u64), vp],
    "GrB_Matrix_nvals": [ctypes.POINTER(u64), vp],
    "GrB_Matrix_wait": [vp, i32],
    "GrM_Matrix_import_CSR": [vp, vp, vp, u64],
    "GrM_Matrix_export_CSR": [vp, vp, vp],
    "GrM_Matrix_build_edges": [vp, vp, vp, u64, ctypes.c_bool],
    "GrB_transpose": [vp, vp, vp, vp, vp],
    "GrM_Matrix_import_dense": [vp, vp, u64, u64],
    "GrM_Matrix_export_dense": [vp, vp],
    "GrB_mxm": [vp, vp, vp, vp, vp, vp, vp],
    "GrM_Matrix_row_degree": [vp, vp],
    "GrM_rmat_edges": [vp, vp, i32, u64, u64, dbl, dbl, dbl],
    "GrM_web_edges": [vp, vp, u64, ctypes.POINTER(u64), u64, u64, ctypes.c_void_p],
    "GrB_mxv": [vp, vp, vp, vp, vp, vp, vp],
    "GrB_Vector_eWiseMult_BinaryOp": [vp, vp, vp, vp, vp, vp, vp],
    "GrB_Vector_eWiseAdd_BinaryOp": [vp, vp, vp, vp, vp, vp, vp],
    "GrB_Vector_apply": [vp, vp, vp, vp, vp, vp],
    "GrB_Vector_apply_BinaryOp1st_FP64": [vp, vp, vp, vp, dbl, vp, vp],
    "GrB_Vector_apply_BinaryOp2nd_FP64": [vp, vp, vp, vp, vp, dbl, vp],
    "GrB_Vector_apply_BinaryOp2nd_Scalar": [vp, vp, vp, vp, vp, vp, vp],
    "GrB_Vector_reduce_Monoid_Scalar": [vp, vp, vp, vp, vp],
    "GrB_Vector_reduce_FP64": [ctypes.POINTER(dbl), vp, vp, vp, vp],
    "GrM_Vector_reduce_masked_Scalar": [vp, vp, vp, vp, vp],
    "GrM_pagerank": [vp, ctypes.POINTER(i32), ctypes.POINTER(dbl), vp, vp, dbl, dbl, i32, i32,
                     vp, i32],
    "GrM_ppr": [vp, ctypes.POINTER(i32), ctypes.POINTER(dbl), vp, vp, vp, dbl, dbl, i32, i32,
                vp, i32],
    "GrM_ppr_batch": [vp, vp, i32, vp, vp, vp, vp, dbl, dbl, i32, i32, i32, ctypes.POINTER(i32),
                      vp, vp],
    "GrM_ppr_stream": [vp, vp, i32, vp, vp, vp, vp, dbl, dbl, i32, i32, i32, i32, vp, vp, vp],
    "GrM_Multigraph_new": [PV, i32, vp],
    "GrM_Multigraph_free": [PV],
    "GrM_Multigraph_offsets": [vp, vp],
    "GrM_pagerank_many": [vp, vp, vp, dbl, dbl, i32, i32, vp, vp],
    "GrM_Matrix_plan_set": [vp, vp, ctypes.c_void_p],
    "GrM_Matrix_plan_get": [ctypes.c_void_p, vp, vp],
    "GrM_autotune_pagerank": [ctypes.c_void_p, ctypes.POINTER(dbl), vp, vp, vp, ctypes.c_char_p],
    "GrM_GNN_new": [PV, vp, u64],
    "GrM_GNN_free": [PV],
    "GrM_GNN_set_params": [vp, vp],
    "GrM_GNN_get_params": [vp, vp],
    "GrM_GNN_get_grad": [vp, vp],
    "GrM_GNN_buffer": [vp, i32, PV, ctypes.POINTER(i64)],
    "GrM_gnn_features": [vp, vp, vp, vp, i32, i32, dbl, u64],
    "GrM_gnn_forward": [vp, vp, vp, ctypes.POINTER(i32)],
    "GrM_gnn_backward": [vp, vp, vp, vp, i64, i32, ctypes.POINTER(dbl)],
    "GrM_gnn_adam_step": [vp, dbl, dbl, dbl, dbl, dbl],
    "GrM_gnn_predict_x0": [vp, vp, vp, vp, vp, i32, i32, dbl, u64, ctypes.POINTER(i32)],
    "GrM_stream_copy": [vp, vp, ctypes.c_size_t],
    "GrM_timing_enable": [ctypes.c_bool],
    "GrM_timing_read": [ctypes.POINTER(dbl), ctypes.POINTER(i64)],
    "GrM_reduce_dense_noalloc": [vp, vp, vp, u64],
}

_lib = None
_lock = threading.Lock()


class GrBError(RuntimeError):
    def __init__(self, info: int, where: str, msg: str):
        self.info = info
        super().__init__("%s returned %s (%d): %s" % (where, _INFO_NAMES.get(info, "?"), info, msg))


def library_path() -> str:
    return LIB_PATH


def load():
    """Load libnbgrb.so; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libnbgrb.so is not built (expected at %s); run "
                "`python paper_2509_14211_amd/build.py` or __graft_entry__.build()" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, args in _FUNCS.items():
            f = getattr(lib, name)
            f.restype = i32
            f.argtypes = args
        lib.GrM_error.restype = ctypes.c_char_p
        lib.GrM_error.argtypes = []
        _lib = lib
        return lib


def builtin(name: str) -> int:
    """Address value held by an exported data symbol (a type or operator)."""
    return vp.in_dll(load(), name).value


def __getattr__(name):  # module-level access to GrB_FP32, GrB_PLUS_FP64, ...
    if name in DATA_SYMBOLS:
        return builtin(name)
    raise AttributeError(name)


def _call(name, *args, ok=(GrB_SUCCESS,)):
    lib = load()
    info = getattr(lib, name)(*args)
    if info not in ok:
        raise GrBError(info, name, lib.GrM_error().decode(errors="replace"))
    return info


def _addr(x) -> int | None:
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


# ---------------------------------------------------------------- context

def GrB_init(mode=GrB_NONBLOCKING):
    _call("GrB_init", mode)


def GrB_finalize():
    _call("GrB_finalize")


def GrM_get_mode() -> int:
    m = i32()
    _call("GrM_get_mode", ctypes.byref(m))
    return m.value


def GrM_set_mode(mode):
    _call("GrM_set_mode", mode)


def GrM_set_stream(stream_handle: int):
    _call("GrM_set_stream", stream_handle)


_ALLOC_T = ctypes.CFUNCTYPE(vp, ctypes.c_size_t, vp)
_FREE_T = ctypes.CFUNCTYPE(None, vp, vp)
_keep = []


def allocator_thunks(alloc, release):
    """C callbacks for GrM_set_allocator around Python callables.  A Python
    exception must not cross into C: ctypes would print it and hand the
    library an undefined (non-null) pointer.  A failed allocation returns
    NULL instead, which the library reports as GrB_OUT_OF_MEMORY."""
    def _alloc(n, ctx):
        try:
            return alloc(n) or None
        except Exception:
            return None

    def _release(p, ctx):
        try:
            release(p)
        except Exception:
            pass

    return _ALLOC_T(_alloc), _FREE_T(_release)


def GrM_set_allocator(alloc=None, release=None):
    """alloc(nbytes) -> int address, release(address) -> None (Python
    callables), or both None for hipMalloc / hipFree."""
    if alloc is None:
        _call("GrM_set_allocator", None, None, None)
        return
    ca, cf = allocator_thunks(alloc, release)
    _keep.append((ca, cf))
    _call("GrM_set_allocator", ctypes.cast(ca, vp), ctypes.cast(cf, vp), None)


def GrM_fail_allocation_after(k: int):
    _call("GrM_fail_allocation_after", k)


def GrM_get_stats() -> dict:
    s = GrM_Stats()
    _call("GrM_get_stats", ctypes.byref(s))
    return {f: getattr(s, f) for f, _ in GrM_Stats._fields_}


def GrM_reset_stats():
    _call("GrM_reset_stats")


def GrM_set_fusion(level: int):
    _call("GrM_set_fusion", level)


def GrM_code_cache_clear():
    _call("GrM_code_cache_clear")


# ---------------------------------------------------------------- vectors with missing entries

GrM_FULL, GrM_BITSET, GrM_SPARSE = 0, 1, 2
_TYPE_SUFFIX = {"FP32": (np.float32, "FP32"), "FP64": (np.float64, "FP64"), "INT32": (np.int32, "INT32")}


def _suffix_of(v) -> str:
    t = GrM_Vector_type(v)
    for name in ("GrB_FP32", "GrB_FP64", "GrB_INT32"):
        if builtin(name) == t:
            return name[4:]
    raise ValueError("vector type has no tuple form")


def GrB_Vector_nvals(v) -> int:
    n = u64()
    _call("GrB_Vector_nvals", ctypes.byref(n), v)
    return int(n.value)


def GrB_Vector_clear(v):
    _call("GrB_Vector_clear", v)


def GrB_Vector_build(w, indices, values, dup=None):
    """w := entries (indices[k], values[k]) from host arrays (w's type)."""
    suf = _suffix_of(w)
    idx = np.ascontiguousarray(indices, dtype=np.uint64)
    val = np.ascontiguousarray(values, dtype=_TYPE_SUFFIX[suf][0])
    if idx.shape != val.shape:
        raise ValueError("indices and values differ in length")
    _call("GrB_Vector_build_" + suf, w, idx.ctypes.data_as(vp), val.ctypes.data_as(vp), len(idx), dup)


def GrB_Vector_extractTuples(v):
    """(indices int64, values) of the present entries, ascending."""
    suf = _suffix_of(v)
    nv = GrB_Vector_nvals(v)
    idx = np.empty(max(nv, 1), dtype=np.uint64)
    val = np.empty(max(nv, 1), dtype=_TYPE_SUFFIX[suf][0])
    n = u64(len(idx))
    _call("GrB_Vector_extractTuples_" + suf, idx.ctypes.data_as(vp), val.ctypes.data_as(vp), ctypes.byref(n), v)
    return idx[:n.value].astype(np.int64), val[:n.value]


def GrB_Vector_assign(w, mask, x, desc=None):
    """w<mask> = x at every position (GrB_ALL)."""
    suf = _suffix_of(w)
    _call("GrB_Vector_assign_" + suf, w, mask, None, x, None, GrB_Vector_size(w), desc)


def GrM_Vector_format(v) -> int:
    f = i32()
    _call("GrM_Vector_format", ctypes.byref(f), v)
    return int(f.value)


def GrM_set_format_policy(policy: int):
    _call("GrM_set_format_policy", policy)


def GrM_set_many_team_max(max_team: int):
    """Largest team of workgroups per graph in later GrM_Multigraph_new calls (1..8)."""
    _call("GrM_set_many_team_max", max_team)


def GrM_set_many_team_wait(ticks: int):
    """Give-up limit of a team barrier wait in 100 MHz ticks (a test hook)."""
    _call("GrM_set_many_team_wait", ticks)


def GrM_error() -> str:
    return load().GrM_error().decode(errors="replace")


# ---------------------------------------------------------------- scalars

def GrB_Scalar_new(type_) -> int:
    h = vp()
    _call("GrB_Scalar_new", ctypes.byref(h), type_)
    return h.value


def GrB_Scalar_free(s):
    h = vp(s)
    _call("GrB_Scalar_free", ctypes.byref(h))


def GrB_Scalar_setElement_FP64(s, x: float):
    _call("GrB_Scalar_setElement_FP64", s, x)


def GrB_Scalar_extractElement_FP64(s):
    """Value of the scalar, or None when it has no value (GrB_NO_VALUE)."""
    x = dbl()
    info = _call("GrB_Scalar_extractElement_FP64", ctypes.byref(x), s, ok=(0, 1))
    return None if info == GrB_NO_VALUE else x.value


def GrB_Scalar_wait(s, mode=GrB_MATERIALIZE):
    _call("GrB_Scalar_wait", s, mode)


def GrM_Scalar_affine(out, alpha, in_, beta):
    _call("GrM_Scalar_affine", out, alpha, in_, beta)


# ---------------------------------------------------------------- vectors

def GrB_Vector_new(type_, n: int) -> int:
    h = vp()
    _call("GrB_Vector_new", ctypes.byref(h), type_, n)
    return h.value


def GrB_Vector_free(v):
    h = vp(v)
    _call("GrB_Vector_free", ctypes.byref(h))


def GrB_Vector_dup(u) -> int:
    h = vp()
    _call("GrB_Vector_dup", ctypes.byref(h), u)
    return h.value


def GrB_Vector_size(v) -> int:
    n = u64()
    _call("GrB_Vector_size", ctypes.byref(n), v)
    return n.value


def GrM_Vector_type(v) -> int:
    t = vp()
    _call("GrM_Vector_type", ctypes.byref(t), v)
    return t.value


def GrB_Vector_wait(v, mode=GrB_MATERIALIZE):
    _call("GrB_Vector_wait", v, mode)


def GrM_Vector_fill(v, value: float):
    _call("GrM_Vector_fill", v, value)


def GrM_Vector_import_dense(v, src, n: int):
    _call("GrM_Vector_import_dense", v, _addr(src), n)


def GrM_Vector_export_dense(dst, n: int, v):
    _call("GrM_Vector_export_dense", _addr(dst), n, v)


def GrM_Vector_device_pointer(v) -> int:
    p = vp()
    _call("GrM_Vector_device_pointer", ctypes.byref(p), v)
    return p.value


# ---------------------------------------------------------------- matrices

def GrB_Matrix_new(type_, nrows: int, ncols: int) -> int:
    h = vp()
    _call("GrB_Matrix_new", ctypes.byref(h), type_, nrows, ncols)
    return h.value


def GrB_Matrix_free(A):
    h = vp(A)
    _call("GrB_Matrix_free", ctypes.byref(h))


def GrB_Matrix_nrows(A) -> int:
    n = u64()
    _call("GrB_Matrix_nrows", ctypes.byref(n), A)
    return n.value


def GrB_Matrix_ncols(A) -> int:
    n = u64()
    _call("GrB_Matrix_ncols", ctypes.byref(n), A)
    return n.value


def GrB_Matrix_nvals(A) -> int:
    n = u64()
    _call("GrB_Matrix_nvals", ctypes.byref(n), A)
    return n.value


def GrB_Matrix_wait(A, mode=GrB_MATERIALIZE):
    _call("GrB_Matrix_wait", A, mode)


def GrM_Matrix_import_CSR(A, rowptr, col, nnz: int):
    _call("GrM_Matrix_import_CSR", A, _addr(rowptr), _addr(col), nnz)


def GrM_Matrix_export_CSR(rowptr, col, A):
    _call("GrM_Matrix_export_CSR", _addr(rowptr), _addr(col), A)


def GrM_Matrix_build_edges(A, src, dst, nedges: int, drop_self: bool = True):
    _call("GrM_Matrix_build_edges", A, _addr(src), _addr(dst), nedges, drop_self)


def GrM_Matrix_import_dense(A, src, nrows: int, ncols: int):
    _call("GrM_Matrix_import_dense", A, _addr(src), nrows, ncols)


def GrM_Matrix_export_dense(dst, A):
    _call("GrM_Matrix_export_dense", _addr(dst), A)


def GrB_mxm(C, Mask, accum, op, A, B, desc=None):
    _call("GrB_mxm", C, Mask, accum, op, A, B, desc)


def GrB_transpose(C, Mask, accum, A, desc=None):
    _call("GrB_transpose", C, Mask, accum, A, desc)


def GrM_Matrix_row_degree(deg, A):
    _call("GrM_Matrix_row_degree", deg, A)


def GrM_rmat_edges(src, dst, scale, nedges, seed, t_a, t_ab, t_abc):
    _call("GrM_rmat_edges", _addr(src), _addr(dst), scale, nedges, seed & (2**64 - 1),
          t_a, t_ab, t_abc)


def GrM_web_edges(src, dst, capacity, n, seed, model) -> int:
    """Web-shaped link list into device arrays src/dst (None, None: only
    count); model is a mapping with the GrM_WebModel fields.  Returns the
    number of links."""
    m = GrM_WebModel(**{f: int(model[f]) for f, _ in GrM_WebModel._fields_})
    cnt = u64()
    _call("GrM_web_edges", _addr(src) if src is not None else None,
          _addr(dst) if dst is not None else None, capacity, ctypes.byref(cnt), n,
          seed & (2**64 - 1), ctypes.addressof(m))
    return int(cnt.value)


# ---------------------------------------------------------------- operations

def GrB_mxv(w, mask, accum, op, A, u, desc=None):
    _call("GrB_mxv", w, mask, accum, op, A, u, desc)


def GrB_Vector_eWiseMult_BinaryOp(w, mask, accum, op, u, v, desc=None):
    _call("GrB_Vector_eWiseMult_BinaryOp", w, mask, accum, op, u, v, desc)


def GrB_Vector_eWiseAdd_BinaryOp(w, mask, accum, op, u, v, desc=None):
    _call("GrB_Vector_eWiseAdd_BinaryOp", w, mask, accum, op, u, v, desc)


def GrB_Vector_apply(w, mask, accum, op, u, desc=None):
    _call("GrB_Vector_apply", w, mask, accum, op, u, desc)


def GrB_Vector_apply_BinaryOp1st_FP64(w, mask, accum, op, s, u, desc=None):
    _call("GrB_Vector_apply_BinaryOp1st_FP64", w, mask, accum, op, s, u, desc)


def GrB_Vector_apply_BinaryOp2nd_FP64(w, mask, accum, op, u, s, desc=None):
    _call("GrB_Vector_apply_BinaryOp2nd_FP64", w, mask, accum, op, u, s, desc)


def GrB_Vector_apply_BinaryOp2nd_Scalar(w, mask, accum, op, u, s, desc=None):
    _call("GrB_Vector_apply_BinaryOp2nd_Scalar", w, mask, accum, op, u, s, desc)


def GrB_Vector_reduce_Monoid_Scalar(s, accum, monoid, u, desc=None):
    _call("GrB_Vector_reduce_Monoid_Scalar", s, accum, monoid, u, desc)


def GrB_Vector_reduce_FP64(accum, monoid, u, desc=None) -> float:
    x = dbl()
    _call("GrB_Vector_reduce_FP64", ctypes.byref(x), accum, monoid, u, desc)
    return x.value


def GrM_Vector_reduce_masked_Scalar(s, mask, monoid, u, desc=None):
    _call("GrM_Vector_reduce_masked_Scalar", s, mask, monoid, u, desc)


def GrM_pagerank(r, AT, outdeg, damping, tol, itermax, dangling=GrM_DANGLING_UNIFORM, x0=None,
                 check_every=8):
    """Returns (iterations, residual); the ranks are left in vector r."""
    it = i32()
    res = dbl()
    _call("GrM_pagerank", r, ctypes.byref(it), ctypes.byref(res), AT, outdeg, damping, tol,
          itermax, dangling, x0, check_every)
    return it.value, res.value


def GrM_Matrix_plan_set(A, type_, cfg: dict | None):
    """cfg: dict with the GrM_PlanConfig fields (missing ones are 0), or None."""
    if cfg is None:
        _call("GrM_Matrix_plan_set", A, type_, None)
        return
    c = GrM_PlanConfig(**cfg)
    _call("GrM_Matrix_plan_set", A, type_, ctypes.addressof(c))


def GrM_Matrix_plan_get(A, type_) -> dict:
    c = GrM_PlanConfig()
    _call("GrM_Matrix_plan_get", ctypes.addressof(c), A, type_)
    return {f: getattr(c, f) for f, _ in GrM_PlanConfig._fields_}


def GrM_autotune_pagerank(AT, outdeg, type_, cache_path: str | None = None):
    """Returns (chosen plan config dict, microseconds per pass or -1 if cached)."""
    c = GrM_PlanConfig()
    us = dbl()
    _call("GrM_autotune_pagerank", ctypes.addressof(c), ctypes.byref(us), AT, outdeg, type_,
          cache_path.encode() if cache_path else None)
    return {f: getattr(c, f) for f, _ in GrM_PlanConfig._fields_}, us.value


def GrM_ppr(r, AT, outdeg, teleport, damping, tol, itermax, dangling=GrM_DANGLING_UNIFORM,
            x0=None, check_every=8):
    """Personalised PageRank; returns (iterations, residual), ranks in r."""
    it = i32()
    res = dbl()
    _call("GrM_ppr", r, ctypes.byref(it), ctypes.byref(res), AT, outdeg, teleport, damping, tol,
          itermax, dangling, x0, check_every)
    return it.value, res.value


def GrM_ppr_batch(X, type_, seed_sets, AT, outdeg, damping, tol, itermax,
                  dangling=GrM_DANGLING_UNIFORM, check_every=8):
    """seed_sets: list of k integer sequences.  X: device buffer (tensor or
    address) of n*k entries of type_ (n x k row-major).  Each column stops
    at its own converged pass.  Returns (passes of the longest-running
    column, per-column converged pass (-1: not within itermax), per-column
    residual at its last pass)."""
    import numpy as np
    k = len(seed_sets)
    ptr = np.zeros(k + 1, dtype=np.int32)
    for q, s in enumerate(seed_sets):
        ptr[q + 1] = ptr[q] + len(s)
    vtx = np.ascontiguousarray(np.concatenate([np.asarray(s, dtype=np.int32) for s in seed_sets])
                               if k else np.zeros(0, np.int32), dtype=np.int32)
    it = i32()
    col_it = np.zeros(max(k, 1), dtype=np.int32)
    col_res = np.zeros(max(k, 1), dtype=np.float64)
    _call("GrM_ppr_batch", _addr(X), type_, k, ptr.ctypes.data, vtx.ctypes.data, AT, outdeg,
          damping, tol, itermax, dangling, check_every, ctypes.byref(it), col_it.ctypes.data,
          col_res.ctypes.data)
    return it.value, col_it[:k].copy(), col_res[:k].copy()


def GrM_ppr_stream(X, type_, seed_sets, AT, outdeg, damping, tol, itermax, dangling=GrM_DANGLING_UNIFORM,
                   k=64, check_every=2):
    """seed_sets: list of integer sequences.  X: device buffer of
    len(seed_sets) * n entries of type_ (set q at offset q * n).  Returns
    per-set (first converged pass, passes run, last residual) numpy arrays."""
    import numpy as np
    q = len(seed_sets)
    ptr = np.zeros(q + 1, dtype=np.int32)
    for i, s in enumerate(seed_sets):
        ptr[i + 1] = ptr[i] + len(s)
    vtx = np.ascontiguousarray(np.concatenate([np.asarray(s, dtype=np.int32) for s in seed_sets])
                               if q else np.zeros(0, np.int32), dtype=np.int32)
    it = np.zeros(max(q, 1), dtype=np.int32)
    ps = np.zeros(max(q, 1), dtype=np.int32)
    res = np.zeros(max(q, 1), dtype=np.float64)
    _call("GrM_ppr_stream", _addr(X), type_, q, ptr.ctypes.data, vtx.ctypes.data, AT, outdeg, damping, tol,
          itermax, dangling, k, check_every, it.ctypes.data, ps.ctypes.data, res.ctypes.data)
    return it[:q].copy(), ps[:q].copy(), res[:q].copy()


def GrM_Multigraph_new(ATs) -> int:
    arr = (ctypes.c_void_p * len(ATs))(*ATs)
    h = vp()
    _call("GrM_Multigraph_new", ctypes.byref(h), len(ATs), ctypes.cast(arr, vp))
    return h.value


def GrM_Multigraph_free(mg):
    h = vp(mg)
    _call("GrM_Multigraph_free", ctypes.byref(h))


def GrM_Multigraph_offsets(mg, ngraphs: int):
    import numpy as np
    off = np.zeros(ngraphs + 1, dtype=np.int64)
    _call("GrM_Multigraph_offsets", off.ctypes.data, mg)
    return off


def GrM_pagerank_many(X, type_, mg, ngraphs: int, damping, tol, itermax,
                      dangling=GrM_DANGLING_UNIFORM):
    """Returns (per-graph passes, per-graph last residual) as numpy arrays."""
    import numpy as np
    it = np.zeros(ngraphs, dtype=np.int32)
    res = np.zeros(ngraphs, dtype=np.float64)
    _call("GrM_pagerank_many", _addr(X), type_, mg, damping, tol, itermax, dangling,
          it.ctypes.data, res.ctypes.data)
    return it, res


def GrM_stream_copy(dst, src, nbytes: int):
    _call("GrM_stream_copy", _addr(dst), _addr(src), nbytes)


def GrM_reduce_dense_noalloc(sum_dev, x_dev, type_, n: int):
    """*sum_dev = sum of x_dev[0:n) (device pointers or tensors), allocating nothing."""
    _call("GrM_reduce_dense_noalloc", _addr(sum_dev), _addr(x_dev) if x_dev is not None else None, type_, n)


def GrM_timing_enable(on: bool):
    _call("GrM_timing_enable", bool(on))


def GrM_timing_read():
    """(total milliseconds, launches) of timed fused passes since the last read."""
    t = dbl()
    n = i64()
    _call("GrM_timing_read", ctypes.byref(t), ctypes.byref(n))
    return t.value, n.value


# ------------------------------------------------------------ warm start

GRM_GNN_NPARAMS = 1601
GNN_BUFFERS = {"counts": 0, "X": 1, "M": 2, "H": 3, "a": 4, "q": 5, "z": 6, "x0": 7, "gq": 8}


def _seeds_i32(seeds):
    import numpy as np
    return np.ascontiguousarray(np.asarray(seeds, dtype=np.int32))


def GrM_GNN_new(act_type, init_seed: int = 0) -> int:
    h = vp()
    _call("GrM_GNN_new", ctypes.byref(h), act_type, init_seed & (2**64 - 1))
    return h.value


def GrM_GNN_free(net):
    h = vp(net)
    _call("GrM_GNN_free", ctypes.byref(h))


def GrM_GNN_set_params(net, theta):
    import numpy as np
    t = np.ascontiguousarray(np.asarray(theta, dtype=np.float32))
    assert t.size == GRM_GNN_NPARAMS
    _call("GrM_GNN_set_params", net, t.ctypes.data)


def GrM_GNN_get_params(net):
    import numpy as np
    t = np.zeros(GRM_GNN_NPARAMS, dtype=np.float32)
    _call("GrM_GNN_get_params", net, t.ctypes.data)
    return t


def GrM_GNN_get_grad(net):
    import numpy as np
    g = np.zeros(GRM_GNN_NPARAMS, dtype=np.float64)
    _call("GrM_GNN_get_grad", net, g.ctypes.data)
    return g


def GrM_GNN_buffer(net, which):
    """(device address, element count) of a work buffer (name or index)."""
    w = GNN_BUFFERS[which] if isinstance(which, str) else int(which)
    p = vp()
    c = i64()
    _call("GrM_GNN_buffer", net, w, ctypes.byref(p), ctypes.byref(c))
    return p.value, c.value


def GrM_gnn_features(net, A, AT, seeds, walkers: int, damping: float, seed: int):
    s = _seeds_i32(seeds)
    _call("GrM_gnn_features", net, A, AT, s.ctypes.data, s.size, walkers, damping, seed & (2**64 - 1))


def GrM_gnn_forward(net, A, AT) -> int:
    """Returns 1 if the prediction fell back to the teleport vector."""
    fb = i32()
    _call("GrM_gnn_forward", net, A, AT, ctypes.byref(fb))
    return fb.value


def GrM_gnn_backward(net, A, AT, x_star, stride: int = 1, accumulate: bool = False) -> float:
    """Gradient of KL(x* || x0) into the network; returns the loss."""
    loss = dbl()
    _call("GrM_gnn_backward", net, A, AT, _addr(x_star), stride, 1 if accumulate else 0, ctypes.byref(loss))
    return loss.value


def GrM_gnn_adam_step(net, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
                      grad_scale: float = 1.0):
    _call("GrM_gnn_adam_step", net, lr, beta1, beta2, eps, grad_scale)


def GrM_gnn_predict_x0(x0, net, A, AT, seeds, walkers: int, damping: float, seed: int) -> int:
    """x0 (a GrB_Vector) = predicted start vector; returns the fallback flag."""
    s = _seeds_i32(seeds)
    fb = i32()
    _call("GrM_gnn_predict_x0", x0, net, A, AT, s.ctypes.data, s.size, walkers, damping, seed & (2**64 - 1),
          ctypes.byref(fb))
    return fb.value
