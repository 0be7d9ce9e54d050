"""Vectors with missing entries on the GPU (sparse / bitset / full storage,
fill-estimate-driven storage and loop drivers) against the reference in
oracle/sparse.py, and the breadth-first search built from them."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import sparse as S

pytestmark = pytest.mark.gpu

OPS = ["plus", "minus", "times", "max", "first", "second", "absdiff"]


def _op(grb, name, t="FP64"):
    return grb.builtin({"plus": "GrB_PLUS", "minus": "GrB_MINUS", "times": "GrB_TIMES", "max": "GrB_MAX",
                        "first": "GrB_FIRST", "second": "GrB_SECOND", "absdiff": "GrM_ABSDIFF"}[name] + "_" + t)


def _new(grb, t, n):
    return grb.GrB_Vector_new(grb.builtin("GrB_" + t), n)


def _from_svec(grb, sv, t="FP64"):
    v = _new(grb, t, sv.n)
    grb.GrB_Vector_build(v, sv.idx, sv.vals)
    return v


def _to_svec(grb, v, n):
    idx, val = grb.GrB_Vector_extractTuples(v)
    return S.SVec(n, idx, val.astype(np.float64))


def _rand(rng, n, fill, integer=True):
    idx = np.nonzero(rng.random(n) < fill)[0]
    vals = rng.integers(-4, 5, len(idx)).astype(np.float64) if integer else rng.normal(size=len(idx))
    return S.SVec(n, idx, vals)


def _same(a, b):
    return np.array_equal(a.idx, b.idx) and np.array_equal(a.vals, b.vals)


@pytest.fixture()
def policy(gpu):
    yield gpu
    gpu.GrM_set_format_policy(0)
    gpu.GrM_set_mode(gpu.GrB_NONBLOCKING)


@pytest.mark.parametrize("t", ["FP32", "FP64", "INT32"])
def test_build_extract_roundtrip(policy, t):
    grb = policy
    rng = np.random.default_rng(1)
    n = 1000
    for pol in (0, 1, 2):
        grb.GrM_set_format_policy(pol)
        idx = rng.choice(n, 40, replace=False)
        vals = rng.integers(-50, 50, 40)
        v = _new(grb, t, n)
        grb.GrB_Vector_build(v, idx, vals)
        assert grb.GrB_Vector_nvals(v) == 40
        got_i, got_v = grb.GrB_Vector_extractTuples(v)
        o = np.argsort(idx)
        assert np.array_equal(got_i, idx[o]) and np.array_equal(got_v, vals[o])
        assert grb.GrM_Vector_format(v) == (grb.GrM_BITSET if pol == 1 else grb.GrM_SPARSE)
        grb.GrB_Vector_clear(v)
        assert grb.GrB_Vector_nvals(v) == 0
        # every entry present -> stored full
        grb.GrB_Vector_build(v, np.arange(n)[::-1], np.arange(n))
        assert grb.GrM_Vector_format(v) == grb.GrM_FULL and grb.GrB_Vector_nvals(v) == n
        grb.GrB_Vector_free(v)


def test_build_duplicates_and_errors(policy):
    grb = policy
    v = _new(grb, "FP64", 10)
    grb.GrB_Vector_build(v, [3, 1, 3, 3], [1.0, 2.0, 4.0, 8.0], dup=_op(grb, "plus"))
    i, x = grb.GrB_Vector_extractTuples(v)
    assert i.tolist() == [1, 3] and x.tolist() == [2.0, 13.0]
    with pytest.raises(grb.GrBError) as e:
        grb.GrB_Vector_build(v, [2, 2], [1.0, 1.0])
    assert e.value.info == grb.GrB_INVALID_VALUE
    with pytest.raises(grb.GrBError) as e:
        grb.GrB_Vector_build(v, [10], [1.0])
    assert e.value.info == grb.GrB_INDEX_OUT_OF_BOUNDS
    # dense-only calls refuse a vector with missing entries
    grb.GrB_Vector_build(v, [1], [1.0])
    out = torch.empty(10, dtype=torch.float64, device="cuda")
    with pytest.raises(grb.GrBError) as e:
        grb.GrM_Vector_export_dense(out, 10, v)
    assert e.value.info == grb.GrB_INVALID_VALUE
    grb.GrB_Vector_free(v)


@pytest.mark.parametrize("fu,fv", [(0.01, 0.3), (0.3, 0.01), (0.02, 0.03), (0.5, 1.0), (1.0, 0.01)])
@pytest.mark.parametrize("pol", [0, 1, 2])
def test_ewise_against_oracle(policy, fu, fv, pol):
    grb = policy
    grb.GrM_set_format_policy(pol)
    rng = np.random.default_rng(int(fu * 1000 + fv * 100 + pol))
    n = 5003
    u, v = _rand(rng, n, fu, integer=False), _rand(rng, n, fv, integer=False)
    gu, gv = _from_svec(grb, u), _from_svec(grb, v)
    w = _new(grb, "FP64", n)
    for op in OPS:
        for add in (False, True):
            f = grb.GrB_Vector_eWiseAdd_BinaryOp if add else grb.GrB_Vector_eWiseMult_BinaryOp
            f(w, None, None, _op(grb, op), gu, gv)
            want = (S.ewise_add if add else S.ewise_mult)(u, v, op)
            assert _same(_to_svec(grb, w, n), want), (op, add)
    for name, k, first in (("minus", 2.5, True), ("times", 3.0, False)):
        if first:
            grb.GrB_Vector_apply_BinaryOp1st_FP64(w, None, None, _op(grb, name), k, gu)
        else:
            grb.GrB_Vector_apply_BinaryOp2nd_FP64(w, None, None, _op(grb, name), gu, k)
        assert _same(_to_svec(grb, w, n), S.apply_bind(u, name, k, first))
    grb.GrB_Vector_apply(w, None, None, grb.builtin("GrB_AINV_FP64"), gu)
    assert _same(_to_svec(grb, w, n), S.apply_unary(u, "ainv"))
    got = grb.GrB_Vector_reduce_FP64(None, grb.builtin("GrB_PLUS_MONOID_FP64"), gu)
    assert abs(got - S.reduce(u)) <= 1e-12 * max(1.0, np.abs(u.vals).sum())
    for h in (gu, gv, w):
        grb.GrB_Vector_free(h)


def test_index_loops_used_for_sparse_inputs(policy):
    grb = policy
    rng = np.random.default_rng(5)
    n = 100000
    u, v = _rand(rng, n, 0.001), _rand(rng, n, 0.5)
    gu, gv = _from_svec(grb, u), _from_svec(grb, v)
    assert grb.GrM_Vector_format(gu) == grb.GrM_SPARSE and grb.GrM_Vector_format(gv) == grb.GrM_BITSET
    w = _new(grb, "FP64", n)
    grb.GrM_reset_stats()
    grb.GrB_Vector_eWiseMult_BinaryOp(w, None, None, _op(grb, "plus"), gv, gu)
    grb.GrB_Vector_wait(w)
    st = grb.GrM_get_stats()
    assert st["index_loops"] == 1 and st["range_loops"] == 0
    assert grb.GrM_Vector_format(w) == grb.GrM_SPARSE
    assert _same(_to_svec(grb, w, n), S.ewise_mult(v, u, "plus"))
    for h in (gu, gv, w):
        grb.GrB_Vector_free(h)


@pytest.fixture(scope="module")
def g10(gpu, oracle_mod):
    from paper_2509_14211_amd import api
    g = api.rmat_graph(10)
    og = oracle_mod.rmat_graph(10)
    yield g, og
    g.free()


@pytest.mark.parametrize("fill", [0.004, 0.2, 1.0])
@pytest.mark.parametrize("mask", [None, "value", "struct", "comp", "struct_comp"])
@pytest.mark.parametrize("replace", [True, False])
def test_masked_mxv_against_oracle(policy, g10, fill, mask, replace):
    """Integer-valued FP64 operands, so sums are exact in any order and
    push and pull must agree bit for bit with the reference."""
    grb = policy
    g, og = g10
    n = g.n
    rng = np.random.default_rng(int(fill * 1000) + (0 if mask is None else len(mask)) + replace)
    u = _rand(rng, n, fill) if fill < 1 else S.SVec.full(rng.integers(-4, 5, n).astype(float))
    gu = _from_svec(grb, u)
    old = _rand(rng, n, 0.3)
    w = _from_svec(grb, old)
    m = _rand(rng, n, 0.4)
    m.vals[::3] = 0.0
    gm = _from_svec(grb, m) if mask else None
    comp = mask in ("comp", "struct_comp")
    struct = mask in ("struct", "struct_comp")
    desc = None
    if mask:
        desc = grb.builtin("GrB_DESC_" + ("R" if replace else "") + ("S" if struct else "") + ("C" if comp else "")) \
            if (replace or struct or comp) else None
    grb.GrM_reset_stats()
    grb.GrB_mxv(w, gm, None, grb.builtin("GrM_PLUS_SECOND_SEMIRING_FP64"), g.AT, gu, desc)
    got = _to_svec(grb, w, n)
    want = S.mxv(og.rowptrT, og.colT, u, m if mask else None, comp, struct, replace or not mask,
                 old if (mask and not replace) else None)
    assert _same(got, want)
    st = grb.GrM_get_stats()
    if fill < 0.01:
        assert st["mxv_push"] == 1
    elif mask or fill < 1:
        assert st["mxv_pull"] == 1
    for h in (gu, w) + ((gm,) if gm else ()):
        grb.GrB_Vector_free(h)


@pytest.fixture(scope="module")
def g_long(gpu, oracle_mod):
    """Rows of A^T longer than the pull mxv's per-group limit (2048 entries,
    summed by a workgroup each): in-hubs 0 and 1 with 5999 and 3000 links,
    among 20,000 random links."""
    from paper_2509_14211_amd import api
    n = 6000
    rng = np.random.default_rng(77)
    src = np.concatenate([np.arange(1, n), np.arange(2, 3002), rng.integers(0, n, 20000)]).astype(np.uint32)
    dst = np.concatenate([np.zeros(n - 1), np.ones(3000), rng.integers(0, n, 20000)]).astype(np.uint32)
    g = api.graph_from_edges(n, src, dst)
    og = oracle_mod.graph_from_edges(n, src, dst)
    assert og.rowptrT[1] - og.rowptrT[0] > 2048 and og.rowptrT[2] - og.rowptrT[1] > 2048
    yield g, og
    g.free()


@pytest.mark.parametrize("fill", [0.2, 1.0])
@pytest.mark.parametrize("mask", [None, "value", "struct_comp"])
@pytest.mark.parametrize("replace", [True, False])
def test_pull_mxv_long_rows_against_oracle(policy, g_long, fill, mask, replace):
    """Pull mxv with rows past the per-group limit: hub 0 lies inside the
    mask and hub 1 outside it (both have old entries), so every mask mode
    sends one long row through the allowed path and one through the
    kept-or-dropped path.  Integer-valued operands: exact in any order."""
    grb = policy
    g, og = g_long
    n = g.n
    rng = np.random.default_rng(int(fill * 10) + (0 if mask is None else len(mask)) + 2 * replace)
    u = _rand(rng, n, fill) if fill < 1 else S.SVec.full(rng.integers(-4, 5, n).astype(float))
    gu = _from_svec(grb, u)
    old = _rand(rng, n, 0.3)
    keep = (old.idx != 0) & (old.idx != 1)
    old = S.SVec(n, np.concatenate([[0, 1], old.idx[keep]]), np.concatenate([[3.0, -2.0], old.vals[keep]]))
    order = np.argsort(old.idx)
    old = S.SVec(n, old.idx[order], old.vals[order])
    w = _from_svec(grb, old)
    m = _rand(rng, n, 0.4)
    mk = (m.idx != 0) & (m.idx != 1)
    m = S.SVec(n, np.concatenate([[0], m.idx[mk]]), np.concatenate([[1.0], m.vals[mk]]))
    order = np.argsort(m.idx)
    m = S.SVec(n, m.idx[order], m.vals[order])
    gm = _from_svec(grb, m) if mask else None
    comp = mask == "struct_comp"
    struct = mask == "struct_comp"
    desc = None
    if mask and (replace or struct or comp):
        desc = grb.builtin("GrB_DESC_" + ("R" if replace else "") + ("S" if struct else "") + ("C" if comp else ""))
    grb.GrM_reset_stats()
    grb.GrB_mxv(w, gm, None, grb.builtin("GrM_PLUS_SECOND_SEMIRING_FP64"), g.AT, gu, desc)
    got = _to_svec(grb, w, n)
    want = S.mxv(og.rowptrT, og.colT, u, m if mask else None, comp, struct, replace or not mask,
                 old if (mask and not replace) else None)
    assert _same(got, want)
    if mask or fill < 1:  # (a full u with no mask takes the dense pass)
        assert grb.GrM_get_stats()["mxv_pull"] == 1
    for h in (gu, w) + ((gm,) if gm else ()):
        grb.GrB_Vector_free(h)


def test_format_policies_give_identical_results(policy, g10):
    """The estimates only choose storage and loop drivers (Section III-D):
    a chain of operations gives the same entries under every policy."""
    grb = policy
    g, og = g10
    n = g.n
    rng = np.random.default_rng(9)
    u, v = _rand(rng, n, 0.01), _rand(rng, n, 0.3)
    results = []
    for pol in (0, 1, 2):
        grb.GrM_set_format_policy(pol)
        gu, gv = _from_svec(grb, u), _from_svec(grb, v)
        w = _new(grb, "FP64", n)
        grb.GrB_mxv(w, gv, None, grb.builtin("GrM_PLUS_SECOND_SEMIRING_FP64"), g.AT, gu,
                    grb.builtin("GrB_DESC_RSC"))
        grb.GrB_Vector_eWiseAdd_BinaryOp(w, None, None, _op(grb, "plus"), w, gu)
        grb.GrB_Vector_apply_BinaryOp2nd_FP64(w, None, None, _op(grb, "times"), w, 2.0)
        s = grb.GrB_Vector_reduce_FP64(None, grb.builtin("GrB_PLUS_MONOID_FP64"), w)
        results.append((_to_svec(grb, w, n), s))
        for h in (gu, gv, w):
            grb.GrB_Vector_free(h)
    for r, s in results[1:]:
        assert _same(r, results[0][0]) and s == results[0][1]
    t = S.mxv(og.rowptrT, og.colT, u, v, True, True, True)
    t = S.apply_bind(S.ewise_add(t, u, "plus"), "times", 2.0, False)
    assert _same(results[0][0], t)


def test_blocking_mode_matches(policy, g10):
    grb = policy
    g, og = g10
    rng = np.random.default_rng(4)
    u = _rand(rng, g.n, 0.02)
    out = []
    for mode in (grb.GrB_NONBLOCKING, grb.GrB_BLOCKING):
        grb.GrM_set_mode(mode)
        gu = _from_svec(grb, u)
        w = _new(grb, "FP64", g.n)
        grb.GrB_mxv(w, None, None, grb.builtin("GrM_PLUS_SECOND_SEMIRING_FP64"), g.AT, gu)
        grb.GrB_Vector_apply(w, None, None, grb.builtin("GrB_ABS_FP64"), w)
        out.append(_to_svec(grb, w, g.n))
        grb.GrB_Vector_free(gu)
        grb.GrB_Vector_free(w)
    assert _same(out[0], out[1])
    assert _same(out[0], S.apply_unary(S.mxv(og.rowptrT, og.colT, u), "abs"))


def test_dense_drivers_reject_missing_entries(policy, g10):
    grb = policy
    g, _ = g10
    deg = _new(grb, "INT32", g.n)
    grb.GrB_Vector_build(deg, [0, 5], [1, 2])
    r = _new(grb, "FP32", g.n)
    with pytest.raises(grb.GrBError) as e:
        grb.GrM_pagerank(r, g.AT, deg, 0.85, 1e-6, 10)
    assert e.value.info == grb.GrB_INVALID_VALUE
    grb.GrB_Vector_free(deg)
    grb.GrB_Vector_free(r)


@pytest.mark.parametrize("scale,sources", [(10, (0, 17, 1023)), (12, (5, 300))])
def test_bfs_against_oracle(policy, oracle_mod, scale, sources):
    from paper_2509_14211_amd import api
    grb = policy
    g = api.rmat_graph(scale)
    og = oracle_mod.rmat_graph(scale)
    try:
        for src in sources:
            grb.GrM_reset_stats()
            lv, depth = api.bfs_levels(g, src)
            got = _to_svec(grb, lv, g.n)
            grb.GrB_Vector_free(lv)
            want = S.bfs_levels(og.rowptrT, og.colT, src)
            assert _same(got, want), src
            st = grb.GrM_get_stats()
            assert st["mxv_push"] + st["mxv_pull"] == depth
    finally:
        g.free()


def test_bfs_unreachable_and_single_vertex(policy):
    from paper_2509_14211_amd import api
    grb = policy
    n, src, dst = synthetic.star_in(8)       # leaves point to the centre
    g = api.graph_from_edges(n, src, dst)
    lv, depth = api.bfs_levels(g, 3)          # leaf 3 reaches only the centre
    i, x = grb.GrB_Vector_extractTuples(lv)
    assert i.tolist() == [0, 3] and x.tolist() == [1, 0] and depth == 2
    grb.GrB_Vector_free(lv)
    lv, depth = api.bfs_levels(g, 0)          # the centre has no out-edge
    i, x = grb.GrB_Vector_extractTuples(lv)
    assert i.tolist() == [0] and x.tolist() == [0] and depth == 1
    grb.GrB_Vector_free(lv)
    g.free()


def test_bfs_scale22_properties(policy):
    """The headline graph: levels checked by the properties that define
    them (source at 0; every edge out of a reached vertex reaches a vertex
    at most one level deeper; every other reached vertex has an in-neighbour
    exactly one level up; nothing else is reached)."""
    from paper_2509_14211_amd import api
    grb = policy
    g = api.rmat_graph(22)
    try:
        rp, col = api.csr_of(g.A)
        rp = rp.cpu().numpy().astype(np.int64)
        col = col.cpu().numpy().astype(np.int64)
        src_of = np.repeat(np.arange(g.n), np.diff(rp))
        deg = np.diff(rp)
        for s in (int(np.argmax(deg)), 12345):
            grb.GrM_reset_stats()
            lv, depth = api.bfs_levels(g, s)
            i, x = grb.GrB_Vector_extractTuples(lv)
            grb.GrB_Vector_free(lv)
            level = np.full(g.n, -1, dtype=np.int64)
            level[i] = x
            assert level[s] == 0
            reached = level >= 0
            e_from = reached[src_of]
            assert np.all(reached[col[e_from]])
            assert np.all(level[col[e_from]] <= level[src_of[e_from]] + 1)
            parent_ok = np.zeros(g.n, dtype=bool)
            tight = e_from & (level[col] == level[src_of] + 1)
            parent_ok[col[tight]] = True
            parent_ok[s] = True
            assert np.all(parent_ok[reached])
            assert depth == level.max() + 1
            st = grb.GrM_get_stats()
            print("bfs from %d: %d reached, depth %d, push %d pull %d" % (
                s, reached.sum(), depth, st["mxv_push"], st["mxv_pull"]), flush=True)
            if reached.sum() > 1000:
                assert st["mxv_push"] >= 1 and st["mxv_pull"] >= 1
    finally:
        g.free()


def test_empty_and_tiny_vectors(policy, g10):
    """Vectors with no entries through every operation, a size-1 vector, and
    assign without a mask (every position, stored full)."""
    grb = policy
    g, og = g10
    n = g.n
    e = _new(grb, "FP64", n)
    grb.GrB_Vector_clear(e)
    u = _from_svec(grb, _rand(np.random.default_rng(2), n, 0.1))
    w = _new(grb, "FP64", n)
    grb.GrB_Vector_eWiseMult_BinaryOp(w, None, None, _op(grb, "plus"), e, u)
    assert grb.GrB_Vector_nvals(w) == 0
    grb.GrB_Vector_eWiseAdd_BinaryOp(w, None, None, _op(grb, "plus"), e, u)
    assert _same(_to_svec(grb, w, n), _to_svec(grb, u, n))
    grb.GrB_Vector_apply(w, None, None, grb.builtin("GrB_ABS_FP64"), e)
    assert grb.GrB_Vector_nvals(w) == 0
    assert grb.GrB_Vector_reduce_FP64(None, grb.builtin("GrB_PLUS_MONOID_FP64"), e) == 0.0
    grb.GrB_mxv(w, None, None, grb.builtin("GrM_PLUS_SECOND_SEMIRING_FP64"), g.AT, e)
    assert grb.GrB_Vector_nvals(w) == 0
    grb.GrB_Vector_assign(w, None, 2.5)
    assert grb.GrM_Vector_format(w) == grb.GrM_FULL and grb.GrB_Vector_nvals(w) == n
    grb.GrB_Vector_assign(w, e, 1.0, grb.builtin("GrB_DESC_R"))   # empty mask + replace: nothing left
    assert grb.GrB_Vector_nvals(w) == 0
    one = _new(grb, "FP32", 1)
    grb.GrB_Vector_build(one, [0], [3.0])
    assert grb.GrM_Vector_format(one) == grb.GrM_FULL
    i, x = grb.GrB_Vector_extractTuples(one)
    assert i.tolist() == [0] and x.tolist() == [3.0]
    for h in (e, u, w, one):
        grb.GrB_Vector_free(h)


def test_push_through_hub_and_empty_rows(policy, oracle_mod):
    """Push from the centre of an out-star (one frontier entry, one long
    column) and from a leaf without out-edges (no entry at all)."""
    from paper_2509_14211_amd import api
    grb = policy
    n, src, dst = synthetic.star_out(5000)
    g = api.graph_from_edges(n, src, dst)
    og = oracle_mod.graph_from_edges(n, src, dst)
    try:
        u = S.SVec(n, [0], [2.0])
        gu = _from_svec(grb, u)
        w = _new(grb, "FP64", n)
        grb.GrM_reset_stats()
        grb.GrB_mxv(w, None, None, grb.builtin("GrM_PLUS_SECOND_SEMIRING_FP64"), g.AT, gu)
        assert _same(_to_svec(grb, w, n), S.mxv(og.rowptrT, og.colT, u))
        assert grb.GrM_get_stats()["mxv_push"] == 1
        v = S.SVec(n, [7], [1.0])                  # a leaf: nothing points out of it
        gv = _from_svec(grb, v)
        grb.GrB_mxv(w, None, None, grb.builtin("GrM_PLUS_SECOND_SEMIRING_FP64"), g.AT, gv)
        assert grb.GrB_Vector_nvals(w) == 0
        for h in (gu, gv, w):
            grb.GrB_Vector_free(h)
    finally:
        g.free()
