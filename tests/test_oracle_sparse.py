"""Pins of the reference for vectors with missing entries (oracle/sparse.py):
brute-force Python sets and dicts on tiny inputs, scipy's sparse product
for mxv, and scipy's shortest-path routine for the breadth-first search
written with these operations."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import synthetic
from oracle import sparse as S


def _rand_svec(rng, n, fill):
    idx = np.nonzero(rng.random(n) < fill)[0]
    return S.SVec(n, idx, rng.normal(size=len(idx)))


def _as_dict(v):
    return {int(i): float(x) for i, x in zip(v.idx, v.vals)}


@pytest.mark.parametrize("seed", range(5))
def test_ewise_against_dicts(seed):
    rng = np.random.default_rng(seed)
    n = 40
    u, v = _rand_svec(rng, n, 0.3), _rand_svec(rng, n, 0.5)
    du, dv = _as_dict(u), _as_dict(v)
    for op in ("plus", "times", "minus", "max", "first", "second", "absdiff"):
        f = S.BINARY[op]
        got = _as_dict(S.ewise_mult(u, v, op))
        assert got.keys() == du.keys() & dv.keys()
        for i in got:
            assert got[i] == f(du[i], dv[i])
        got = _as_dict(S.ewise_add(u, v, op))
        assert got.keys() == du.keys() | dv.keys()
        for i in got:
            want = f(du[i], dv[i]) if (i in du and i in dv) else du.get(i, dv.get(i))
            assert got[i] == want
    assert S.reduce(u) == pytest.approx(sum(du.values()), abs=1e-12)
    assert S.reduce(S.SVec.empty(n)) == 0.0
    a = _as_dict(S.apply_bind(u, "minus", 2.5, first=True))
    assert a == {i: 2.5 - x for i, x in du.items()}
    assert _as_dict(S.apply_unary(u, "ainv")) == {i: -x for i, x in du.items()}


def _rand_graph(rng, n, m):
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    A = sp.csr_matrix((np.ones(m), (src, dst)), shape=(n, n))
    A.data[:] = 1.0
    A.sum_duplicates()
    A.data[:] = 1.0
    A.sort_indices()
    return A


@pytest.mark.parametrize("fill", [0.0, 0.05, 0.4, 1.0])
def test_mxv_against_scipy(fill):
    """Values: the pattern product with scipy on the present entries;
    presence: rows meeting at least one present entry (all rows when u is
    full)."""
    rng = np.random.default_rng(7)
    n = 300
    A = _rand_graph(rng, n, 1500)
    u = _rand_svec(rng, n, fill) if fill < 1 else S.SVec.full(rng.normal(size=n))
    w = S.mxv(A.indptr, A.indices, u)
    pres = (A @ u.present().astype(float)) > 0
    if fill == 1.0:
        pres[:] = True
    assert np.array_equal(w.present(), pres)
    np.testing.assert_allclose(w.dense(), A @ u.dense(), rtol=1e-12, atol=1e-12)


def test_mask_semantics():
    rng = np.random.default_rng(3)
    n = 200
    A = _rand_graph(rng, n, 800)
    u = _rand_svec(rng, n, 0.2)
    plain = _as_dict(S.mxv(A.indptr, A.indices, u))
    old = _rand_svec(rng, n, 0.5)
    mask = _rand_svec(rng, n, 0.4)
    mask.vals[::3] = 0.0  # present zeros: value mask false, structural true
    for comp in (False, True):
        for structural in (False, True):
            for replace in (False, True):
                got = _as_dict(S.mxv(A.indptr, A.indices, u, mask, comp, structural, replace, old))
                allowed = {i for i in range(n)
                           if (i in _as_dict(mask) and (structural or _as_dict(mask)[i] != 0)) != comp}
                want = {i: x for i, x in plain.items() if i in allowed}
                if not replace:
                    want.update({i: x for i, x in _as_dict(old).items() if i not in allowed})
                assert got == want
    # complement of an empty mask = no mask
    got = S.mxv(A.indptr, A.indices, u, S.SVec.empty(n), comp=True, structural=True)
    assert _as_dict(got) == plain
    lv = S.assign_scalar(old, n, 7.0, mask=mask, structural=True)
    want = _as_dict(old)
    want.update({int(i): 7.0 for i in mask.idx})
    assert _as_dict(lv) == want


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_bfs_against_scipy_shortest_path(oracle_mod, seed):
    """Levels equal the unweighted shortest-path distances from the source;
    unreachable vertices have no entry."""
    rng = np.random.default_rng(seed)
    n = 400
    A = _rand_graph(rng, n, 700)
    AT = A.T.tocsr()
    AT.sort_indices()
    src = int(rng.integers(0, n))
    lv = S.bfs_levels(AT.indptr, AT.indices, src)
    dist = shortest_path(A, method="D", unweighted=True, directed=True, indices=src)
    reach = np.isfinite(dist)
    assert np.array_equal(lv.present(), reach)
    assert np.array_equal(lv.dense()[reach], dist[reach])


def test_bfs_closed_forms():
    # directed path 0 -> 1 -> ... -> 9: level i at vertex i
    n = 10
    A = sp.csr_matrix((np.ones(n - 1), (np.arange(n - 1), np.arange(1, n))), shape=(n, n))
    AT = A.T.tocsr()
    lv = S.bfs_levels(AT.indptr, AT.indices, 0)
    assert np.array_equal(lv.idx, np.arange(n)) and np.array_equal(lv.vals, np.arange(n))
    lv = S.bfs_levels(AT.indptr, AT.indices, 5)
    assert np.array_equal(lv.idx, np.arange(5, n))
    # out-star: centre at level 0, every leaf at level 1
    n, src, dst = synthetic.star_out(6)
    A = sp.csr_matrix((np.ones(len(src)), (src, dst)), shape=(n, n))
    AT = A.T.tocsr()
    lv = S.bfs_levels(AT.indptr, AT.indices, 0)
    assert _as_dict(lv) == {0: 0.0, **{i: 1.0 for i in range(1, n)}}
