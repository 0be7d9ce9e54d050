"""GrB_mxm restricted to a CSR pattern times a dense matrix (at most 64
columns), and the dense import/export it needs, through the C ABI.

Every column of the product is the oracle's plus-second mxv of that column
(oracle/sparse.py, itself pinned against scipy's sparse product).  FP64
entries agree within 1e-12 of the sum of the absolute terms; FP32 entries
within (row length) * 2^-24 of it, the bound of recursive FP32 summation
(the kernel's sums are shorter chains, so the bound holds for any order)."""
import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu


def _oracle_product(rowptr, col, B):
    from oracle import sparse
    cols = [sparse.mxv(rowptr, col, sparse.SVec.full(B[:, c])).dense() for c in range(B.shape[1])]
    absB = np.abs(B)
    mag = np.stack([sparse.mxv(rowptr, col, sparse.SVec.full(absB[:, c])).dense() for c in range(B.shape[1])], 1)
    return np.stack(cols, 1), mag


def _mxm(grb, A, nrows, B: torch.Tensor, dtype_name):
    typ = grb.builtin(dtype_name)
    k = B.shape[1]
    Bm = grb.GrB_Matrix_new(typ, B.shape[0], k)
    grb.GrM_Matrix_import_dense(Bm, B.contiguous(), B.shape[0], k)
    C = grb.GrB_Matrix_new(typ, nrows, k)
    sfx = "FP64" if dtype_name == "GrB_FP64" else "FP32"
    grb.GrB_mxm(C, None, None, grb.builtin("GrM_PLUS_SECOND_SEMIRING_" + sfx), A, Bm, None)
    out = torch.empty(nrows, k, dtype=B.dtype, device="cuda")
    grb.GrM_Matrix_export_dense(out, C)
    assert grb.GrB_Matrix_nvals(C) == nrows * k
    grb.GrB_Matrix_free(C)
    grb.GrB_Matrix_free(Bm)
    return out.cpu().numpy().astype(np.float64)


def _check(got, ref, mag, rowlen, dtype):
    if dtype == torch.float64:
        bound = 1e-12 * mag + 1e-300
    else:
        bound = (np.maximum(rowlen, 1)[:, None] * 2.0 ** -24 + 2.0 ** -24) * mag + 1e-30
    assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
# k <= 16 runs the packed pass (lane groups of 4, 8 or 16 columns, several
# entries per load): each group width at and past its edge
@pytest.mark.parametrize("k", [1, 4, 5, 7, 8, 9, 16, 17, 64])
def test_mxm_rmat_against_oracle(nonblocking, oracle_mod, dtype, k):
    from paper_2509_14211_amd import api
    grb = nonblocking
    print("mxm rmat scale 11 k", k, dtype, flush=True)
    g = api.rmat_graph(11)
    og = oracle_mod.rmat_graph(11)
    n = g.n
    B = np.stack([synthetic.random_vector(n, 100 + c) for c in range(k)], 1)
    Bt = torch.from_numpy(B).to(dtype).cuda()
    Bq = Bt.cpu().numpy().astype(np.float64)  # the values the GPU multiplies
    got = _mxm(grb, g.AT, n, Bt, "GrB_FP64" if dtype == torch.float64 else "GrB_FP32")
    ref, mag = _oracle_product(og.rowptrT, og.colT, Bq)
    _check(got, ref, mag, np.diff(og.rowptrT), dtype)
    g.free()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_mxm_hub_rows_and_rectangular(nonblocking, oracle_mod, dtype):
    """Rows longer than a tile (split into chunks and finished by the last
    wavefront), empty rows, and a rectangular pattern."""
    from paper_2509_14211_amd import api
    grb = nonblocking
    name = "GrB_FP64" if dtype == torch.float64 else "GrB_FP32"
    # inward star: row 0 of A^T holds 20000 entries
    spec = synthetic.star_in(20000)
    g = api.graph_from_edges(*spec)
    og = oracle_mod.graph_from_edges(*spec)
    k = 5
    B = np.stack([synthetic.random_vector(g.n, 300 + c) for c in range(k)], 1)
    Bt = torch.from_numpy(B).to(dtype).cuda()
    got = _mxm(grb, g.AT, g.n, Bt, name)
    ref, mag = _oracle_product(og.rowptrT, og.colT, Bt.cpu().numpy().astype(np.float64))
    _check(got, ref, mag, np.diff(og.rowptrT), dtype)
    g.free()
    # rectangular 700 x 3000 pattern from a random edge list
    nr, nc = 700, 3000
    rng = np.random.default_rng(5)
    src = rng.integers(0, nr, 20000)
    dst = rng.integers(0, nc, 20000)
    keys = np.unique(src.astype(np.int64) * nc + dst)
    rows, cols = keys // nc, keys % nc
    rowptr = np.zeros(nr + 1, dtype=np.int32)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    col = cols.astype(np.int32)
    A = grb.GrB_Matrix_new(grb.builtin(name), nr, nc)
    grb.GrM_Matrix_import_CSR(A, torch.from_numpy(rowptr).cuda(), torch.from_numpy(col).cuda(), len(col))
    k = 33
    B = np.stack([synthetic.random_vector(nc, 400 + c) for c in range(k)], 1)
    Bt = torch.from_numpy(B).to(dtype).cuda()
    got = _mxm(grb, A, nr, Bt, name)
    ref, mag = _oracle_product(rowptr, col, Bt.cpu().numpy().astype(np.float64))
    _check(got, ref, mag, np.diff(rowptr), dtype)
    grb.GrB_Matrix_free(A)


def test_mxm_errors(nonblocking):
    from paper_2509_14211_amd import api
    grb = nonblocking
    g = api.rmat_graph(8)
    n = g.n
    f32, f64 = grb.builtin("GrB_FP32"), grb.builtin("GrB_FP64")
    sem = grb.builtin("GrM_PLUS_SECOND_SEMIRING_FP32")
    B = grb.GrB_Matrix_new(f32, n, 4)
    grb.GrM_Matrix_import_dense(B, torch.ones(n, 4, device="cuda"), n, 4)
    C = grb.GrB_Matrix_new(f32, n, 4)
    with pytest.raises(grb.GrBError) as e:       # a mask
        grb.GrB_mxm(C, g.AT, None, sem, g.AT, B, None)
    assert e.value.info == -8
    C64 = grb.GrB_Matrix_new(f64, n, 4)
    with pytest.raises(grb.GrBError) as e:       # output type
        grb.GrB_mxm(C64, None, None, sem, g.AT, B, None)
    assert e.value.info == -5
    C3 = grb.GrB_Matrix_new(f32, n, 3)
    with pytest.raises(grb.GrBError) as e:       # output shape
        grb.GrB_mxm(C3, None, None, sem, g.AT, B, None)
    assert e.value.info == -6
    B65 = grb.GrB_Matrix_new(f32, n, 65)
    grb.GrM_Matrix_import_dense(B65, torch.ones(n, 65, device="cuda"), n, 65)
    C65 = grb.GrB_Matrix_new(f32, n, 65)
    with pytest.raises(grb.GrBError) as e:       # more than 64 columns
        grb.GrB_mxm(C65, None, None, sem, g.AT, B65, None)
    assert e.value.info == -8
    with pytest.raises(grb.GrBError) as e:       # a pattern where dense values are expected
        grb.GrB_mxm(C, None, None, sem, g.AT, g.A, None)
    assert e.value.info == -8
    w = api.vector_from_tensor(torch.zeros(n, device="cuda"))
    u = api.vector_from_tensor(torch.zeros(4, device="cuda"))
    with pytest.raises(grb.GrBError) as e:       # a dense matrix where a pattern is expected
        grb.GrB_mxv(w, None, None, sem, B, u, None)
    assert e.value.info == -3
    grb.GrB_Vector_free(w)
    grb.GrB_Vector_free(u)
    with pytest.raises(grb.GrBError) as e:
        grb.GrM_Matrix_export_dense(torch.empty(n, n, device="cuda"), g.AT)
    assert e.value.info == -3
    with pytest.raises(grb.GrBError) as e:       # partial import
        grb.GrM_Matrix_import_dense(B, torch.ones(n, 4, device="cuda"), n - 1, 4)
    assert e.value.info == -6
    grb.GrB_mxm(C, None, None, sem, g.AT, B, None)
    out = torch.empty(n, 4, device="cuda")
    grb.GrM_Matrix_export_dense(out, C)
    indeg = torch.diff(api.csr_of(g.AT)[0]).float()
    assert torch.equal(out, indeg[:, None].expand(n, 4))
    for h in (B, C, C64, C3, B65, C65):
        grb.GrB_Matrix_free(h)
    g.free()
