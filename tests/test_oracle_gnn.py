"""Pins of the warm-start oracle (oracle/gnn.py) against facts that do not
come from that code: the C oracle's SplitMix64 stream, walks that are
deterministic, the personalised PageRank iterates of the C oracle, a dense
matrix product, permutation equivariance, finite differences and Adam's
closed form on a constant gradient."""
import numpy as np
import pytest

import oracle
import synthetic
from oracle import gnn


def _graph(edges_fn, *a):
    n, src, dst = edges_fn(*a)
    return oracle.graph_from_edges(n, src, dst)


def test_splitmix_matches_c_oracle():
    keys = np.array([0, 1, 2, 3, 1000, 2 ** 20 + 7, 2 ** 40 + 3], dtype=np.uint64)
    for seed in (0, 1, 1234567, 2 ** 63 + 5):
        got = gnn.splitmix64(seed, keys)
        want = [oracle.splitmix64(seed, int(k)) for k in keys]
        assert [int(x) for x in got] == want


def test_walks_on_cycle_without_restart_are_rotations():
    # damping 1: no restart; every vertex has out-degree 1, so walker w sits
    # at seeds[w mod |S|] + t after t steps
    n = 10
    g = _graph(synthetic.cycle, n)
    seeds = [2, 7]
    W = 37
    c = gnn.walk_counts(g, seeds, W, 1.0, seed=5)
    for t in range(1, gnn.STEPS + 1):
        want = np.zeros(n, dtype=np.int64)
        for w in range(W):
            want[(seeds[w % 2] + t) % n] += 1
        assert np.array_equal(c[t - 1], want)


def test_walks_restart_at_dangling_vertex():
    # path 0 -> 1 from seed 0, no random restart: 1, then restart to 0, ...
    g = _graph(synthetic.path2)
    c = gnn.walk_counts(g, [0], 16, 1.0, seed=9)
    for t in range(1, gnn.STEPS + 1):
        assert c[t - 1][0 if t % 2 == 0 else 1] == 16


def test_walks_with_certain_restart_stay_on_seeds():
    n, src, dst = synthetic.random_edges(50, 300, seed=3)
    g = oracle.graph_from_edges(n, src, dst)
    seeds = [4, 9, 31]
    c = gnn.walk_counts(g, seeds, 999, 0.0, seed=11)
    off = np.ones(n, dtype=bool)
    off[seeds] = False
    assert np.all(c[:, off] == 0)
    assert np.all(c.sum(axis=1) == 999)


def test_walk_distribution_matches_ppr_iterates():
    # After t steps the walkers sample the t-th iterate of the personalised
    # PageRank map started at the teleport vector.  With |S| dividing W the
    # start is exactly uniform on S; the L1 error of a W-sample estimate of
    # an n-point distribution is at most sqrt(n / W) in expectation.
    g = oracle.rmat_graph(8)
    seeds = [3, 17, 100, 200]
    W = 1 << 16
    d = 0.85
    c = gnn.walk_counts(g, seeds, W, d, seed=77)
    bound = 2.0 * np.sqrt(g.n / W)
    for t in range(1, gnn.STEPS + 1):
        xt = oracle.ppr(g, seeds, d, fixed_iters=t).x
        err = np.abs(c[t - 1] / W - xt).sum()
        assert err < bound, (t, err, bound)


def test_features_on_inward_star():
    # leaves 1..5 point at the centre 0
    g = _graph(synthetic.star_in, 5)
    X = gnn.features(g, [2], 64, 0.85, seed=1)
    assert X.shape == (6, gnn.NF)
    assert X[0, 1] == pytest.approx(np.log(6.0)) and X[0, 2] == 0.0
    assert np.allclose(X[1:, 1], 0.0) and np.allclose(X[1:, 2], np.log(2.0))
    assert X[2, 0] == 1.0 and X[:, 0].sum() == 1.0


def test_mean_aggregation_matches_dense_product():
    n, src, dst = synthetic.random_edges(40, 200, seed=8)
    g = oracle.graph_from_edges(n, src, dst)
    Y = np.random.default_rng(0).normal(size=(n, 5))
    A = np.zeros((n, n))
    rp = np.asarray(g.rowptr)
    for u in range(n):
        A[u, np.asarray(g.col)[rp[u]:rp[u + 1]]] = 1.0
    indeg = A.sum(axis=0)
    want = (A.T @ Y) / np.maximum(indeg, 1)[:, None]
    assert np.allclose(gnn.mean_in(g, Y), want, rtol=1e-13, atol=1e-13)


def test_forward_is_permutation_equivariant():
    n, src, dst = synthetic.random_edges(30, 120, seed=4)
    g = oracle.graph_from_edges(n, src, dst)
    rng = np.random.default_rng(1)
    X = rng.normal(size=(n, gnn.NF))
    theta = gnn.init_params(3) + 0.05 * rng.normal(size=gnn.NPARAMS)
    perm = rng.permutation(n)  # vertex v becomes perm[v]
    gp = oracle.graph_from_edges(n, perm[src], perm[dst])
    Xp = np.empty_like(X)
    Xp[perm] = X
    z = gnn.forward(g, theta, X)["z"]
    zp = gnn.forward(gp, theta, Xp)["z"]
    assert np.allclose(zp[perm], z, rtol=1e-12, atol=1e-12)


def test_z_at_matches_forward():
    n, src, dst = synthetic.random_edges(40, 160, seed=12)
    g = oracle.graph_from_edges(n, src, dst)
    rng = np.random.default_rng(4)
    X = rng.normal(size=(n, gnn.NF))
    theta = gnn.init_params(5) + 0.05 * rng.normal(size=gnn.NPARAMS)
    z = gnn.forward(g, theta, X)["z"]
    vs = [0, 3, 17, 39]
    assert np.allclose(gnn.z_at(g, theta, lambda u: X[u], vs), z[vs], rtol=1e-12, atol=1e-12)


def test_softmax_kl_gradient_identity():
    rng = np.random.default_rng(2)
    z = rng.normal(size=9)
    xs = rng.random(9)
    xs[3] = 0.0
    xs /= xs.sum()
    h = 1e-6
    fd = np.array([(gnn.kl_loss(xs, gnn.softmax(z + h * e)) - gnn.kl_loss(xs, gnn.softmax(z - h * e))) / (2 * h)
                   for e in np.eye(9)])
    assert np.allclose(fd, gnn.softmax(z) - xs, rtol=1e-6, atol=1e-9)
    assert gnn.kl_loss(xs, xs) == pytest.approx(0.0, abs=1e-15)


def test_backward_matches_central_differences():
    n, src, dst = synthetic.random_edges(12, 40, seed=6)
    g = oracle.graph_from_edges(n, src, dst)
    rng = np.random.default_rng(5)
    X = rng.normal(size=(n, gnn.NF))
    xs = rng.random(n)
    xs /= xs.sum()
    theta = gnn.init_params(7) + 0.1 * rng.normal(size=gnn.NPARAMS)
    # keep every pre-activation away from the ReLU kink
    pre = gnn.forward(g, theta, X)["pre"]
    assert np.abs(pre).min() > 1e-4
    loss, grad = gnn.backward(g, theta, X, xs)
    h = 1e-6
    fd = np.empty(gnn.NPARAMS)
    for i in range(gnn.NPARAMS):
        e = np.zeros(gnn.NPARAMS)
        e[i] = h
        lp = gnn.kl_loss(xs, gnn.softmax(gnn.forward(g, theta + e, X)["z"]))
        lm = gnn.kl_loss(xs, gnn.softmax(gnn.forward(g, theta - e, X)["z"]))
        fd[i] = (lp - lm) / (2 * h)
    assert loss == pytest.approx(gnn.kl_loss(xs, gnn.softmax(gnn.forward(g, theta, X)["z"])))
    scale = np.abs(grad).max()
    assert np.abs(fd - grad).max() <= 1e-6 * scale


def test_adam_constant_gradient_moves_by_lr():
    theta, m, v = np.array([1.0]), np.zeros(1), np.zeros(1)
    g = np.array([0.3])
    for t in range(1, 6):
        prev = theta.copy()
        theta, m, v = gnn.adam_step(theta, g, m, v, t, lr=0.01, eps=1e-8)
        assert prev[0] - theta[0] == pytest.approx(0.01 * 0.3 / (0.3 + 1e-8), rel=1e-12)


def test_predict_falls_back_to_teleport_on_nan():
    g = _graph(synthetic.cycle, 6)
    theta = gnn.init_params(0)
    theta[0] = np.nan
    x0, fell = gnn.predict_x0(g, theta, [1, 4], 64, 0.85, 3)
    assert fell and np.allclose(x0, [0, 0.5, 0, 0, 0.5, 0])
    x0, fell = gnn.predict_x0(g, gnn.init_params(0), [1, 4], 64, 0.85, 3)
    assert not fell and x0.sum() == pytest.approx(1.0)
