"""Smaller entry points of the C ABI on the GPU: mode query, matrix
dimensions and waits, scalar waits, the device pointer of a vector, the
fused-pass timer, and the allocation-failure hook (a failed allocation
returns GrB_OUT_OF_MEMORY and leaves the library usable)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def test_mode_and_matrix_queries(nonblocking):
    from paper_2509_14211_amd import api
    grb = nonblocking
    assert grb.GrM_get_mode() == grb.GrB_NONBLOCKING
    grb.GrM_set_mode(grb.GrB_BLOCKING)
    assert grb.GrM_get_mode() == grb.GrB_BLOCKING
    grb.GrM_set_mode(grb.GrB_NONBLOCKING)
    g = api.rmat_graph(8)
    assert grb.GrB_Matrix_nrows(g.AT) == 256 and grb.GrB_Matrix_ncols(g.AT) == 256
    grb.GrB_Matrix_wait(g.AT)
    g.free()


def test_scalar_wait_and_device_pointer(nonblocking):
    from paper_2509_14211_amd import api
    grb = nonblocking
    x = torch.arange(1, 1001, dtype=torch.float64, device="cuda")
    v = api.vector_from_tensor(x)
    s = grb.GrB_Scalar_new(grb.builtin("GrB_FP64"))
    grb.GrB_Vector_reduce_Monoid_Scalar(s, None, grb.builtin("GrB_PLUS_MONOID_FP64"), v)
    grb.GrB_Scalar_wait(s)
    assert grb.GrB_Scalar_extractElement_FP64(s) == 500500.0
    p = grb.GrM_Vector_device_pointer(v)
    assert p != 0
    assert torch.equal(api.device_copy(p, 1000, torch.float64), x)
    sp = grb.GrB_Vector_new(grb.builtin("GrB_FP64"), 1000)
    grb.GrB_Vector_build(sp, [3], [1.0])
    with pytest.raises(grb.GrBError) as e:
        grb.GrM_Vector_device_pointer(sp)
    assert e.value.info == grb.GrB_INVALID_VALUE
    for h in (v, sp):
        grb.GrB_Vector_free(h)
    grb.GrB_Scalar_free(s)


def test_fused_pass_timer(nonblocking):
    from paper_2509_14211_amd import api
    grb = nonblocking
    g = api.rmat_graph(12)
    grb.GrM_timing_read()  # drop earlier records
    grb.GrM_timing_enable(True)
    try:
        _, it, _ = api.pagerank(g, torch.float32, 0.85, 0.0, 5)
        ms, launches = grb.GrM_timing_read()
        assert launches == 5 and ms > 0.0
    finally:
        grb.GrM_timing_enable(False)
        g.free()


def test_allocation_failure_is_reported_and_recoverable(blocking):
    from paper_2509_14211_amd import api
    grb = blocking
    n = 123457  # a size no earlier test allocated, so the buffer cache cannot serve it
    a = api.vector_from_tensor(torch.ones(n, dtype=torch.float64, device="cuda"))
    b = api.vector_from_tensor(torch.full((n,), 2.0, dtype=torch.float64, device="cuda"))
    w = grb.GrB_Vector_new(grb.builtin("GrB_FP64"), n)
    grb.GrM_fail_allocation_after(1)
    try:
        with pytest.raises(grb.GrBError) as e:
            grb.GrB_Vector_eWiseAdd_BinaryOp(w, None, None, grb.builtin("GrB_PLUS_FP64"), a, b)
        assert e.value.info == grb.GrB_OUT_OF_MEMORY
    finally:
        grb.GrM_fail_allocation_after(0)
    grb.GrB_Vector_eWiseAdd_BinaryOp(w, None, None, grb.builtin("GrB_PLUS_FP64"), a, b)
    out = api.tensor_from_vector(w, torch.float64)
    assert torch.all(out == 3.0)
    for h in (a, b, w):
        grb.GrB_Vector_free(h)
