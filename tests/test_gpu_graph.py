"""GPU graph input (R-MAT edges, CSR build, out-degree, transpose) against
the oracle: integer work, so bit-exact."""
import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("scale,seed", [(1, 3), (10, 10), (14, 14)])
def test_rmat_edges_bitwise(gpu, oracle_mod, scale, seed):
    from paper_2509_14211_amd import api
    print("rmat scale", scale, flush=True)
    src, dst = api.rmat_device_edges(scale, 16, seed)
    osrc, odst = oracle_mod.rmat_edges(scale, 16, seed)
    assert np.array_equal(_np(src).view(np.uint32), osrc)
    assert np.array_equal(_np(dst).view(np.uint32), odst)


def _check_graph(g, og):
    from paper_2509_14211_amd import api
    rp, col = api.csr_of(g.A)
    assert np.array_equal(_np(rp), og.rowptr)
    assert np.array_equal(_np(col), og.col)
    rpT, colT = api.csr_of(g.AT)
    assert np.array_equal(_np(rpT), og.rowptrT)
    assert np.array_equal(_np(colT), og.colT)
    deg = api.tensor_from_vector(g.outdeg, torch.int32)
    assert np.array_equal(_np(deg), og.outdeg)


@pytest.mark.parametrize("scale", [10, 13])
def test_rmat_graph_bitwise(gpu, oracle_mod, scale):
    from paper_2509_14211_amd import api
    print("graph scale", scale, flush=True)
    g = api.rmat_graph(scale)
    og = oracle_mod.rmat_graph(scale)
    assert g.m == og.m
    _check_graph(g, og)
    g.free()


@pytest.mark.parametrize("n,ne,seed,drop", [(1, 4, 1, True), (7, 50, 2, False), (300, 9000, 3, True),
                                            (5000, 20000, 4, False)])
def test_edge_list_build_bitwise(gpu, oracle_mod, n, ne, seed, drop):
    from paper_2509_14211_amd import api
    n, src, dst = synthetic.random_edges(n, ne, seed)
    g = api.graph_from_edges(n, src, dst, drop)
    og = oracle_mod.graph_from_edges(n, src, dst, drop)
    _check_graph(g, og)
    g.free()


def test_empty_edge_list(gpu):
    from paper_2509_14211_amd import api
    g = api.graph_from_edges(5, np.zeros(0, np.uint32), np.zeros(0, np.uint32))
    rp, col = api.csr_of(g.A)
    assert np.array_equal(_np(rp), np.zeros(6, np.int32)) and col.numel() == 0
    assert g.m == 0
    g.free()


def test_out_of_range_edge_rejected(gpu):
    from paper_2509_14211_amd import api, grb
    with pytest.raises(grb.GrBError) as e:
        api.graph_from_edges(4, np.array([0, 1], np.uint32), np.array([1, 4], np.uint32))
    assert e.value.info == -105


def test_import_csr_validation(gpu):
    from paper_2509_14211_amd import grb
    A = grb.GrB_Matrix_new(grb.builtin("GrB_FP32"), 3, 3)
    good_rp = torch.tensor([0, 1, 1, 2], dtype=torch.int32, device="cuda")
    good_col = torch.tensor([2, 0], dtype=torch.int32, device="cuda")
    grb.GrM_Matrix_import_CSR(A, good_rp, good_col, 2)
    assert grb.GrB_Matrix_nvals(A) == 2
    bad_col = torch.tensor([3, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(grb.GrBError) as e:
        grb.GrM_Matrix_import_CSR(A, good_rp, bad_col, 2)
    assert e.value.info == -3
    bad_rp = torch.tensor([0, 2, 1, 2], dtype=torch.int32, device="cuda")
    with pytest.raises(grb.GrBError):
        grb.GrM_Matrix_import_CSR(A, bad_rp, good_col, 2)
    assert grb.GrB_Matrix_nvals(A) == 2  # unchanged after a rejected import
    grb.GrB_Matrix_free(A)
