"""Nonblocking GraphBLAS PageRank for AMD Instinct MI355X (gfx950).

The product is libnbgrb.so (C ABI in include/nbgrb.h, HIP kernels in
csrc/).  ``grb`` binds it with the C names; ``api`` adds torch plumbing
(stream, caching allocator, tensor copies).
"""
from . import grb  # noqa: F401

__all__ = ["grb"]
