"""Personalised PageRank on the GPU: the single-vector driver (GrM_ppr) and
the batched SpMM driver (GrM_ppr_batch), each column against the FP64
oracle at the same pass count."""
import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu

D = 0.85


def _tcode(grb, dtype):
    return grb.builtin("GrB_FP32" if dtype == torch.float32 else "GrB_FP64")


def _ppr_single(grb, g, seeds, dtype, **kw):
    from paper_2509_14211_amd import api
    n = g.n
    v = torch.zeros(n, dtype=dtype, device="cuda")
    v[torch.as_tensor(seeds, dtype=torch.long)] = 1.0 / len(seeds)
    vv = api.vector_from_tensor(v)
    r = grb.GrB_Vector_new(_tcode(grb, dtype), n)
    it, res = grb.GrM_ppr(r, g.AT, g.outdeg, vv, D, kw.get("tol", 1e-9), kw.get("itermax", 1000),
                          kw.get("dangling", 1), None, 8)
    x = api.tensor_from_vector(r, dtype).cpu().numpy().astype(np.float64)
    grb.GrB_Vector_free(r)
    grb.GrB_Vector_free(vv)
    return x, it, res


def _batch(grb, g, sets, dtype, tol, itermax=1000, dangling=1):
    X = torch.empty(g.n * len(sets), dtype=dtype, device="cuda")
    it, col_it, col_res = grb.GrM_ppr_batch(X, _tcode(grb, dtype), sets, g.AT, g.outdeg, D, tol,
                                            itermax, dangling)
    return X.view(g.n, len(sets)).cpu().numpy().astype(np.float64), it, col_it, col_res


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("relabel", [0, 1])
def test_ppr_single_matches_oracle(nonblocking, oracle_mod, mode, relabel):
    from paper_2509_14211_amd import api
    grb = nonblocking
    g = api.rmat_graph(12)
    og = oracle_mod.rmat_graph(12)
    for dtype in (torch.float64, torch.float32):
        grb.GrM_Matrix_plan_set(g.AT, _tcode(grb, dtype),
                                dict(kernel=1, lds_entries=512, lds_rows=256, long_row=512, chunk=512,
                                     grid=0, hot=1 << 20, relabel=relabel))
    for seeds in synthetic.ppr_seed_sets(g.n, 3, seed=11):
        x, it, res = _ppr_single(grb, g, seeds, torch.float64, dangling=mode)
        ref = oracle_mod.ppr(og, seeds, D, fixed_iters=it, mode=mode)
        assert np.abs(x - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12
        free = oracle_mod.ppr(og, seeds, D, tol=1e-9, mode=mode)
        assert abs(it - free.iters) <= 1
        x, it, res = _ppr_single(grb, g, seeds, torch.float32, tol=1e-6, dangling=mode)
        ref = oracle_mod.ppr(og, seeds, D, fixed_iters=it, mode=mode)
        assert np.abs(x - ref.x).sum() <= 1e-5
    g.free()


@pytest.mark.parametrize("relabel", [0, 1])
@pytest.mark.parametrize("k", [1, 7, 64])
def test_ppr_batch_matches_oracle(nonblocking, oracle_mod, k, relabel):
    from paper_2509_14211_amd import api
    grb = nonblocking
    print("ppr batch k", k, "relabel", relabel, flush=True)
    g = api.rmat_graph(11)
    og = oracle_mod.rmat_graph(11)
    for dtype in (torch.float64, torch.float32):
        grb.GrM_Matrix_plan_set(g.AT, _tcode(grb, dtype),
                                dict(kernel=1, lds_entries=512, lds_rows=256, long_row=512, chunk=512,
                                     grid=0, hot=0, relabel=relabel))
    sets = synthetic.ppr_seed_sets(g.n, k, seed=7)
    X, it, col_it, col_res = _batch(grb, g, sets, torch.float64, tol=1e-9)
    # each column stops at its own converged pass (the slowest sets the
    # batch's pass count); once half the columns have stopped the product
    # narrows, so the spread below exercises the narrowed passes
    print("converged passes", sorted(col_it.tolist()), flush=True)
    assert it >= 1 and col_res.max() <= 1e-9 and it == col_it.max()
    for q, s in enumerate(sets):
        ref = oracle_mod.ppr(og, s, D, fixed_iters=int(col_it[q]))
        assert np.abs(X[:, q] - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12, q
        assert abs(col_res[q] - ref.resid) <= 1e-12, q
        free = oracle_mod.ppr(og, s, D, tol=1e-9)
        assert abs(int(col_it[q]) - free.iters) <= 1, (q, col_it[q], free.iters)
    X, it, col_it, _ = _batch(grb, g, sets, torch.float32, tol=1e-6)
    for q, s in enumerate(sets):
        ref = oracle_mod.ppr(og, s, D, fixed_iters=int(col_it[q]))
        assert np.abs(X[:, q] - ref.x).sum() <= 1e-5, q
    g.free()


def test_ppr_batch_columns_stop_independently(nonblocking, oracle_mod):
    """Sets that converge at very different passes: a seed on a vertex
    without in- or out-links converges after one pass, a set on the hub
    much later.  Each column equals the oracle after its own pass count,
    whether the batch had narrowed by then or not."""
    from paper_2509_14211_amd import api
    grb = nonblocking
    m = 400
    n, src, dst = synthetic.star_both(m)
    # vertices m+1 .. m+40: isolated
    n2 = n + 40
    g = api.graph_from_edges(n2, src, dst)
    og = oracle_mod.graph_from_edges(n2, src, dst)
    sets = [[n + i] for i in range(30)] + [[0], [1, 2], list(range(3, 40))]
    for dangling in (1, 0):
        X, it, col_it, col_res = _batch(grb, g, sets, torch.float64, tol=1e-13, dangling=dangling)
        print("converged passes", col_it.tolist(), flush=True)
        assert len(set(col_it.tolist())) > 1
        for q, s in enumerate(sets):
            ref = oracle_mod.ppr(og, s, D, fixed_iters=int(col_it[q]), mode=dangling)
            assert np.abs(X[:, q] - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12, (dangling, q)
            free = oracle_mod.ppr(og, s, D, tol=1e-13, mode=dangling)
            assert abs(int(col_it[q]) - free.iters) <= 1, (dangling, q, col_it[q], free.iters)
    g.free()


def test_ppr_batch_drop_mode_and_hubs(nonblocking, oracle_mod):
    """DROP mode, and a hub row longer than a chunk (split across wavefronts)."""
    from paper_2509_14211_amd import api
    grb = nonblocking
    n, src, dst = synthetic.star_both(3000)
    g = api.graph_from_edges(n, src, dst)
    og = oracle_mod.graph_from_edges(n, src, dst)
    sets = [[0], [1, 2, 3], list(range(5, 21))]
    X, it, col_it, _ = _batch(grb, g, sets, torch.float64, tol=1e-12, dangling=0)
    for q, s in enumerate(sets):
        ref = oracle_mod.ppr(og, s, D, fixed_iters=int(col_it[q]), mode=0)
        assert np.abs(X[:, q] - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12
    g.free()


def test_ppr_batch_all_vertices_is_global_pagerank(nonblocking):
    from paper_2509_14211_amd import api
    grb = nonblocking
    g = api.rmat_graph(10)
    X, it, col_it, _ = _batch(grb, g, [list(range(g.n))], torch.float64, tol=1e-10)
    x, it2, _ = api.pagerank(g, torch.float64, tol=1e-10)
    assert it == it2 == col_it[0]
    assert np.abs(X[:, 0] - x.cpu().numpy()).sum() <= 1e-13
    g.free()


def test_ppr_batch_invariants_and_errors(nonblocking):
    from paper_2509_14211_amd import api
    grb = nonblocking
    g = api.rmat_graph(10)
    sets = synthetic.ppr_seed_sets(g.n, 5, seed=3)
    X, it, _, _ = _batch(grb, g, sets, torch.float64, tol=1e-8)
    rp, _ = api.csr_of(g.AT)
    indeg = np.diff(rp.cpu().numpy())
    for q, s in enumerate(sets):
        assert abs(X[:, q].sum() - 1.0) < 1e-12
        zero = indeg == 0
        zero[s] = False
        assert np.all(X[zero, q] == 0.0)
    Xb = torch.empty(g.n * 2, dtype=torch.float64, device="cuda")
    t = grb.builtin("GrB_FP64")
    for bad in ([[1], []], [[1, 1]], [[g.n]], [[-1]]):
        with pytest.raises(grb.GrBError):
            grb.GrM_ppr_batch(Xb, t, bad, g.AT, g.outdeg, D, 1e-6, 100)
    with pytest.raises(grb.GrBError):
        grb.GrM_ppr_batch(Xb, t, [[0]] * 65, g.AT, g.outdeg, D, 1e-6, 100)
    X, it, col_it, _ = _batch(grb, g, sets, torch.float64, tol=2.0)
    assert it == 0 and np.all(col_it == -1)
    g.free()


def _stream(grb, g, sets, dtype, tol, k, check_every=2, itermax=1000, dangling=1):
    X = torch.zeros(len(sets) * g.n, dtype=dtype, device="cuda")
    it, ps, res = grb.GrM_ppr_stream(X, _tcode(grb, dtype), [list(map(int, s)) for s in sets], g.AT, g.outdeg, D,
                                     tol, itermax, dangling, k, check_every)
    return X.reshape(len(sets), g.n).cpu().numpy().astype(np.float64), it, ps, res


@pytest.mark.parametrize("k,relabel", [(64, 1), (7, 0)])
def test_ppr_stream_matches_oracle(nonblocking, oracle_mod, k, relabel):
    """More seed sets than column slots: each set's ranks equal the oracle's
    after the passes it ran, its first converged pass matches a free oracle
    solve, and slots are reused (sets > k)."""
    from paper_2509_14211_amd import api
    grb = nonblocking
    print("ppr stream k", k, "relabel", relabel, flush=True)
    g = api.rmat_graph(11)
    og = oracle_mod.rmat_graph(11)
    for dtype in (torch.float64, torch.float32):
        grb.GrM_Matrix_plan_set(g.AT, _tcode(grb, dtype),
                                dict(kernel=1, lds_entries=512, lds_rows=256, long_row=512, chunk=512,
                                     grid=0, hot=0, relabel=relabel))
    sets = synthetic.ppr_seed_sets(g.n, 150, seed=21)
    X, it, ps, res = _stream(grb, g, sets, torch.float64, 1e-9, k, check_every=3)
    # a set stops at its converged pass (frozen there until written out)
    assert np.all(it >= 1) and np.all(it == ps) and res.max() <= 1e-9
    for q, s in enumerate(sets):
        ref = oracle_mod.ppr(og, s, D, fixed_iters=int(ps[q]))
        assert np.abs(X[q] - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12, q
        free = oracle_mod.ppr(og, s, D, tol=1e-9)
        assert abs(int(it[q]) - free.iters) <= 1, (q, it[q], free.iters)
    X, it, ps, res = _stream(grb, g, sets, torch.float32, 1e-6, k)
    for q, s in enumerate(sets):
        ref = oracle_mod.ppr(og, s, D, fixed_iters=int(ps[q]))
        assert np.abs(X[q] - ref.x).sum() <= 1e-5, q
    g.free()


def test_ppr_stream_itermax_and_drop_mode(nonblocking, oracle_mod):
    """Sets that cannot converge retire after exactly itermax passes."""
    from paper_2509_14211_amd import api
    grb = nonblocking
    n, src, dst = synthetic.star_both(3000)
    g = api.graph_from_edges(n, src, dst)
    og = oracle_mod.graph_from_edges(n, src, dst)
    sets = [[0], [1, 2, 3], list(range(5, 21)), [7], [2999]]
    X, it, ps, res = _stream(grb, g, sets, torch.float64, 1e-14, 2, check_every=4, itermax=5, dangling=0)
    assert np.all(ps == 5) and np.all(it == -1)
    for q, s in enumerate(sets):
        ref = oracle_mod.ppr(og, s, D, fixed_iters=5, mode=0)
        assert np.abs(X[q] - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12
    with pytest.raises(grb.GrBError):
        _stream(grb, g, [[1, 1]], torch.float64, 1e-9, 2)
    g.free()
