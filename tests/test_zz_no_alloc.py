"""The allocation-free sum GrM_reduce_dense_noalloc through the C ABI: its
result equals GrB_Vector_reduce_FP64's on the same values bit for bit (same
kernel and summation order), on two calls in a row with the second input
smaller than the first (the shared static scratch keeps the first call's
partials), and the calls hand out no device buffer at all."""
import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu


def _reference(grb, api, x):
    v = api.vector_from_tensor(x)
    try:
        return grb.GrB_Vector_reduce_FP64(None, grb.builtin("GrB_PLUS_MONOID_FP64"), v)
    finally:
        grb.GrB_Vector_free(v)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_sum_matches_reduce(nonblocking, dtype):
    from paper_2509_14211_amd import api
    grb = nonblocking
    tname = "GrB_FP32" if dtype == torch.float32 else "GrB_FP64"
    # several workgroups' worth with a ragged tail, then a smaller input
    sizes = [3_000_017, 70_001]
    inputs = [torch.from_numpy(synthetic.random_vector(n, seed=40 + k)).to(dtype).cuda()
              for k, n in enumerate(sizes)]
    refs = [_reference(grb, api, x) for x in inputs]
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    before = grb.GrM_get_stats()["device_allocs"]
    for k, x in enumerate(inputs):
        print("noalloc sum: %s n=%d call %d" % (tname, x.numel(), k), flush=True)
        grb.GrM_reduce_dense_noalloc(out[k:k + 1], x, grb.builtin(tname), x.numel())
    torch.cuda.synchronize()
    assert grb.GrM_get_stats()["device_allocs"] == before
    got = out.cpu().numpy()
    for k, x in enumerate(inputs):
        assert got[k] == refs[k], (k, got[k], refs[k])
        exact = float(np.sum(x.cpu().numpy().astype(np.float64)))
        assert abs(got[k] - exact) <= 1e-12 * float(np.sum(np.abs(x.cpu().numpy().astype(np.float64))))


def test_noalloc_sum_edge_cases(nonblocking):
    grb = nonblocking
    out = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    grb.GrM_reduce_dense_noalloc(out, None, grb.builtin("GrB_FP64"), 0)
    torch.cuda.synchronize()
    assert out.item() == 0.0
    one = torch.tensor([2.5], dtype=torch.float64, device="cuda")
    grb.GrM_reduce_dense_noalloc(out, one, grb.builtin("GrB_FP64"), 1)
    torch.cuda.synchronize()
    assert out.item() == 2.5
    with pytest.raises(grb.GrBError) as e:
        grb.GrM_reduce_dense_noalloc(out, one, grb.builtin("GrB_INT32"), 1)
    assert e.value.info == grb.GrB_DOMAIN_MISMATCH
    with pytest.raises(grb.GrBError) as e:
        grb.GrM_reduce_dense_noalloc(out, one, grb.builtin("GrB_FP64"), (1 << 40) + 1)
    assert e.value.info == grb.GrB_INVALID_VALUE
    with pytest.raises(grb.GrBError) as e:
        grb.GrM_reduce_dense_noalloc(out, None, grb.builtin("GrB_FP64"), 5)
    assert e.value.info == grb.GrB_NULL_POINTER
