"""Pins of the oracle's PageRank (Fig. 6 loop, blocking, FP64).

The oracle is checked against things it does not compute itself:
  * a dense LU solve (LAPACK gesv via numpy) of the linear system whose
    fixed point the iteration converges to, built from a dense adjacency
    matrix made directly from the edge list;
  * closed forms on hand graphs (cycle, complete digraph, empty graph,
    three kinds of star, a 2-vertex path, a single vertex), derived by hand;
  * invariants that hold at any size (mass conservation, the DROP mass
    recursion, positivity, equal rank on zero-in-degree vertices, the
    contraction of the residual).
Each check is chosen so that a plausible slip in the oracle -- a dropped
teleport or dangling term, a wrong damping placement, a transposed
operand, an off-by-one in the loop control -- makes at least one fail.
"""
import numpy as np
import pytest

import synthetic

D = 0.85


def _dense_system(n, src, dst, mode, v):
    """(M, b) with M x = b the fixed point equation, from the raw edge list."""
    A = np.zeros((n, n))
    for s, t in zip(src.tolist(), dst.tolist()):
        if s != t:
            A[s, t] = 1.0
    outdeg = A.sum(axis=1)
    dinv = np.where(outdeg > 0, 1.0 / np.where(outdeg > 0, outdeg, 1), 0.0)
    P = A.T * dinv[None, :]           # P[i, j] = 1/outdeg_j for j -> i
    M = np.eye(n) - D * P
    if mode == 1:
        dang = (outdeg == 0).astype(float)
        M = M - D * np.outer(v, dang)
    return M, (1 - D) * v


def _graph(oracle_mod, spec):
    n, src, dst = spec
    return oracle_mod.graph_from_edges(n, src, dst), src, dst


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("scale", [3, 5, 7, 9])
def test_pagerank_matches_dense_lu(oracle_mod, mode, scale):
    src, dst = oracle_mod.rmat_edges(scale, 16, 100 + scale)
    n = 1 << scale
    g = oracle_mod.graph_from_edges(n, src, dst)
    v = np.full(n, 1.0 / n)
    M, b = _dense_system(n, src, dst, mode, v)
    x_lu = np.linalg.solve(M, b)
    r = oracle_mod.pagerank(g, D, fixed_iters=400, mode=mode)
    assert r.iters == 400
    rel = np.abs(r.x - x_lu).sum() / np.abs(x_lu).sum()
    assert rel <= 1e-12


@pytest.mark.parametrize("mode", [0, 1])
def test_ppr_matches_dense_lu(oracle_mod, mode):
    scale = 8
    n = 1 << scale
    src, dst = oracle_mod.rmat_edges(scale, 16, 321)
    g = oracle_mod.graph_from_edges(n, src, dst)
    seeds = synthetic.ppr_seed_sets(n, 3, seed=5)
    for s in seeds:
        v = oracle_mod.teleport_vector(n, s)
        M, b = _dense_system(n, src, dst, mode, v)
        x_lu = np.linalg.solve(M, b)
        r = oracle_mod.ppr(g, s, D, fixed_iters=400, mode=mode)
        assert np.abs(r.x - x_lu).sum() / np.abs(x_lu).sum() <= 1e-12


def test_hand_graph_lu(oracle_mod):
    """A non-R-MAT graph with dangling vertices, a self-loop and duplicates."""
    n = 6
    src = np.array([0, 0, 1, 2, 2, 3, 3, 3, 4, 0], np.uint32)
    dst = np.array([1, 2, 2, 0, 0, 3, 4, 1, 1, 5], np.uint32)
    g = oracle_mod.graph_from_edges(n, src, dst)
    for mode in (0, 1):
        M, b = _dense_system(n, src, dst, mode, np.full(n, 1.0 / n))
        r = oracle_mod.pagerank(g, D, tol=0.0, itermax=300, mode=mode)
        assert np.allclose(r.x, np.linalg.solve(M, b), rtol=1e-13, atol=0)


# ------------------------------------------------------------------ closed forms

def _solve(oracle_mod, spec, mode, **kw):
    g, _, _ = _graph(oracle_mod, spec)
    kw.setdefault("tol", 0.0)
    kw.setdefault("itermax", 300)
    return g, oracle_mod.pagerank(g, D, mode=mode, **kw)


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("make", [lambda: synthetic.cycle(17), lambda: synthetic.complete(9)])
def test_uniform_fixed_point_graphs(oracle_mod, mode, make):
    n = make()[0]
    g, r = _solve(oracle_mod, make(), mode, tol=1e-12, itermax=50)
    # no dangling vertices: both modes give 1/n, reached in one pass
    assert r.iters == 1
    assert np.allclose(r.x, 1.0 / n, rtol=1e-14, atol=0)


def test_empty_graph(oracle_mod):
    n = 10
    _, r = _solve(oracle_mod, synthetic.empty(n), 1)
    assert np.allclose(r.x, 1.0 / n, rtol=1e-14, atol=0)
    _, r = _solve(oracle_mod, synthetic.empty(n), 0)
    assert np.allclose(r.x, (1 - D) / n, rtol=1e-14, atol=0)


def test_single_vertex(oracle_mod):
    _, r = _solve(oracle_mod, synthetic.empty(1), 1)
    assert abs(r.x[0] - 1.0) < 1e-15


@pytest.mark.parametrize("m", [1, 4, 31])
def test_star_both_ways(oracle_mod, m):
    n = m + 1
    _, r = _solve(oracle_mod, synthetic.star_both(m), 1)
    xc = (1 + D * m) / (n * (1 + D))
    xl = (D + m) / (m * n * (1 + D))
    assert abs(r.x[0] - xc) <= 1e-14 * xc
    assert np.allclose(r.x[1:], xl, rtol=1e-13, atol=0)
    # from the uniform start the residual is exactly 2 (m-1) d^t / n
    _, r = _solve(oracle_mod, synthetic.star_both(m), 1, itermax=30)
    t = np.arange(1, 31)
    want = 2 * (m - 1) * D ** t / n
    assert np.allclose(r.rho_hist, want, rtol=1e-10, atol=1e-16)


@pytest.mark.parametrize("m", [1, 5, 40])
def test_star_inward(oracle_mod, m):
    n = m + 1
    _, r = _solve(oracle_mod, synthetic.star_in(m), 1)
    assert abs(r.x[0] - (1 + m * D) / (m + 1 + m * D)) < 1e-14
    assert np.allclose(r.x[1:], 1 / (m + 1 + m * D), rtol=1e-13, atol=0)
    _, r = _solve(oracle_mod, synthetic.star_in(m), 0)
    assert abs(r.x[0] - (1 - D) * (1 + m * D) / n) < 1e-14
    assert np.allclose(r.x[1:], (1 - D) / n, rtol=1e-13, atol=0)


@pytest.mark.parametrize("m", [1, 5, 40])
def test_star_outward(oracle_mod, m):
    n = m + 1
    _, r = _solve(oracle_mod, synthetic.star_out(m), 1)
    assert abs(r.x[0] - 1 / (n + D)) < 1e-14
    assert np.allclose(r.x[1:], (m + D) / (m * (n + D)), rtol=1e-13, atol=0)
    _, r = _solve(oracle_mod, synthetic.star_out(m), 0)
    assert abs(r.x[0] - (1 - D) / n) < 1e-14
    assert np.allclose(r.x[1:], (1 - D) * (1 + D / m) / n, rtol=1e-13, atol=0)


def test_path2(oracle_mod):
    _, r = _solve(oracle_mod, synthetic.path2(), 1)
    assert np.allclose(r.x, [1 / (2 + D), (1 + D) / (2 + D)], rtol=1e-14, atol=0)


# ------------------------------------------------------------------ loop control

def test_loop_control(oracle_mod):
    g = oracle_mod.rmat_graph(9)
    r = oracle_mod.pagerank(g, D, tol=1e-6, itermax=1000)
    # stops at the first pass whose residual is <= tol, not one later
    assert r.rho_hist[-1] <= 1e-6 and np.all(r.rho_hist[:-1] > 1e-6)
    assert r.resid == r.rho_hist[-1]
    r2 = oracle_mod.pagerank(g, D, tol=1e-6, itermax=3)
    assert r2.iters == 3 and r2.resid > 1e-6
    r3 = oracle_mod.pagerank(g, D, tol=1e-6, fixed_iters=5)
    assert r3.iters == 5
    assert np.array_equal(r3.rho_hist, r.rho_hist[:5])
    # tolerance at or above the initial residual of 1: no pass at all
    r4 = oracle_mod.pagerank(g, D, tol=1.0, itermax=10)
    assert r4.iters == 0 and np.allclose(r4.x, 1.0 / g.n)


# ------------------------------------------------------------------ invariants

@pytest.mark.parametrize("scale", [10, 12])
def test_invariants_uniform(oracle_mod, scale):
    g = oracle_mod.rmat_graph(scale)
    n = g.n
    for k in (1, 2, 7, 20):
        r = oracle_mod.pagerank(g, D, fixed_iters=k, mode=1)
        assert abs(r.x.sum() - 1.0) <= 64 * n * np.finfo(float).eps
        c_k = (1 - D) / n + D * r.D_hist[k - 1] / n
        assert np.all(r.x >= (1 - D) / n * (1 - 1e-12))
        zero_in = g.indeg == 0
        assert zero_in.any()
        # zero-in-degree vertices hold only the teleport term, all equal
        assert np.all(r.x[zero_in] == r.x[zero_in][0])
        assert abs(r.x[zero_in][0] - c_k) <= 1e-15 * c_k
        # D_k is the mass on dangling vertices
        assert abs(r.D_hist[k] - r.x[g.outdeg == 0].sum()) <= 1e-13
    r = oracle_mod.pagerank(g, D, fixed_iters=40, mode=1)
    rho = r.rho_hist
    assert np.all(rho[1:] <= D * rho[:-1] * (1 + 1e-9) + 1e-15)


def test_invariants_drop(oracle_mod):
    g = oracle_mod.rmat_graph(10)
    r = oracle_mod.pagerank(g, D, fixed_iters=12, mode=0)
    # mass recursion of the paper's variant: S_{k+1} = d (S_k - D_k) + (1-d)
    S = [1.0]
    for k in range(1, 13):
        rk = oracle_mod.pagerank(g, D, fixed_iters=k, mode=0)
        S.append(rk.x.sum())
    for k in range(12):
        assert abs(S[k + 1] - (D * (S[k] - r.D_hist[k]) + (1 - D))) < 1e-13
    assert r.x.sum() < 1.0


def test_ppr_invariants(oracle_mod):
    g = oracle_mod.rmat_graph(10)
    sets = synthetic.ppr_seed_sets(g.n, 4, seed=7)
    for s in sets:
        r = oracle_mod.ppr(g, s, D, fixed_iters=15)
        assert abs(r.x.sum() - 1.0) < 1e-12
        nonseed_zero_in = (g.indeg == 0)
        nonseed_zero_in[s] = False
        assert np.all(r.x[nonseed_zero_in] == 0.0)
    # seed set = all vertices reduces to global PageRank
    r_all = oracle_mod.ppr(g, np.arange(g.n), D, fixed_iters=10)
    r_glob = oracle_mod.pagerank(g, D, fixed_iters=10)
    assert np.allclose(r_all.x, r_glob.x, rtol=1e-13, atol=0)


def test_threads_do_not_change_bits(oracle_mod):
    g = oracle_mod.rmat_graph(12)
    oracle_mod.set_threads(1)
    a = oracle_mod.pagerank(g, D, fixed_iters=8)
    oracle_mod.set_threads(4)
    b = oracle_mod.pagerank(g, D, fixed_iters=8)
    assert np.array_equal(a.x, b.x) and np.array_equal(a.rho_hist, b.rho_hist)
