"""Pins of the oracle's web-shaped generator (the stand-in for the web crawl
of the paper's Section IV).

The generator is defined link by link from a counter-based stream; these
checks pin it to what its definition implies without re-evaluating that
definition: the closed-form law of the out-degrees, the exact shape of each
kind of link in models that emit only that kind, the tails of the distance
and popularity laws, the affine relabelling of global links, degenerate
models, and agreement between the whole-graph and the one-row forms.
"""
from fractions import Fraction

import numpy as np
import pytest

import synthetic

MODEL = synthetic.WEB_MODEL


def _model(**kw):
    m = dict(MODEL)
    m.update(kw)
    return m


def _pareto_tail(c, x):
    """P(floor(c 2^52 / X) >= x) for X uniform on 1..2^52."""
    if x <= c:
        return Fraction(1)
    return Fraction((c << 52) // x, 1 << 52)


def test_web_degree_law(oracle_mod):
    """k_u = 0 with probability p_zero / 2^16, else min(kmax, D(kmin)) with
    P(D >= x) = floor(kmin 2^52 / x) / 2^52: sample mean, variance share,
    the zero fraction and the capped fraction within 5 sigma."""
    n = 1 << 18
    deg = oracle_mod.web_degrees(n, 11, MODEL)
    kmin, kmax, pz = MODEL["kmin"], MODEL["kmax"], Fraction(MODEL["p_zero"], 65536)
    tail = [_pareto_tail(kmin, x) for x in range(1, kmax + 1)]
    mean = (1 - pz) * sum(tail)
    second = (1 - pz) * sum((2 * x - 1) * t for x, t in zip(range(1, kmax + 1), tail))
    var = float(second - mean * mean)
    assert abs(deg.mean() - float(mean)) < 5 * np.sqrt(var / n)
    p0 = float(pz)
    assert abs((deg == 0).mean() - p0) < 5 * np.sqrt(p0 * (1 - p0) / n)
    pc = float((1 - pz) * tail[-1])
    assert abs((deg == kmax).mean() - pc) < 5 * np.sqrt(pc / n)
    assert deg[deg > 0].min() == kmin and deg.max() == kmax


def test_web_links_in_vertex_order(oracle_mod):
    n = 3000
    src, dst = oracle_mod.web_edges(n, 5, MODEL)
    deg = oracle_mod.web_degrees(n, 5, MODEL)
    assert len(src) == deg.sum()
    assert np.all(np.diff(src.astype(np.int64)) >= 0)
    assert np.array_equal(np.bincount(src, minlength=n), deg)
    assert dst.max() < n


def test_web_degenerate_models(oracle_mod):
    src, dst = oracle_mod.web_edges(500, 3, _model(p_zero=65536))
    assert len(src) == 0
    deg = oracle_mod.web_degrees(500, 3, _model(p_zero=0, kmin=5, kmax=5))
    assert np.all(deg == 5)


def test_web_home_links_clear_low_bits(oracle_mod):
    """With only home links every target is u with its low h bits cleared,
    h uniform on 6..21.  Vertices whose low 21 bits are all ones expose h
    exactly: u - v = 2^h - 1."""
    n = 1 << 24
    model = _model(p_zero=0, p_home=65536, p_local=0, kmin=4000, kmax=4000)
    us = [(k << 21) | ((1 << 21) - 1) for k in range(8)]
    hs = []
    for u in us:
        v = oracle_mod.web_row_links(n, 21, model, u).astype(np.int64)
        diff = u - v
        h = np.log2(diff + 1)
        assert np.all(h == np.round(h))
        hs.append(np.round(h).astype(int))
    hs = np.concatenate(hs)
    assert hs.min() >= 6 and hs.max() <= 21
    freq = np.bincount(hs, minlength=22)[6:] / len(hs)
    sigma = np.sqrt((1 / 16) * (15 / 16) / len(hs))
    assert np.all(np.abs(freq - 1 / 16) < 5 * sigma)
    # any vertex: the target is an aligned block front at or below u
    src, dst = oracle_mod.web_edges(1 << 12, 4, _model(p_zero=0, p_home=65536, p_local=0))
    s, d = src.astype(np.int64), dst.astype(np.int64)
    assert np.all(d <= s) and np.all(d % 64 == 0) and np.all(s - d < (1 << 21))


def test_web_local_distance_law(oracle_mod):
    """Only local links, k_u = 50 > local_min: distances are at least 50,
    P(d >= x) = floor(50 2^52 / x) / 2^52, and each direction has half."""
    n = 1 << 22
    model = _model(p_zero=0, p_home=0, p_local=65536, kmin=50, kmax=50, local_min=16)
    src, dst = oracle_mod.web_edges(1 << 13, 8, model)
    s, d = src.astype(np.int64), dst.astype(np.int64)
    # generate on the big vertex range so no distance wraps: rows of the
    # first 2^13 vertices of an n = 2^22 graph
    fwd = []
    for u in range(0, 1 << 13, 7):
        v = oracle_mod.web_row_links(n, 8, model, u).astype(np.int64)
        fwd.append((v - u) % n)
    f = np.concatenate(fwd)
    back = f > n // 2
    dist = np.where(back, n - f, f)
    # a draw beyond n - 1 is capped there, i.e. one step the other way
    capped = dist == 1
    assert np.all(capped | (dist >= 50)) and capped.mean() < 1e-3
    dist, back = dist[~capped], back[~capped]
    N = len(dist)
    for x in (100, 500, 5000):
        p = float(_pareto_tail(50, x))
        assert abs((dist >= x).mean() - p) < 5 * np.sqrt(p * (1 - p) / N)
    assert abs(back.mean() - 0.5) < 5 * np.sqrt(0.25 / N)
    # small graph: the same law modulo n never yields a self-loop
    assert np.all(s != d)


def test_web_global_popularity_and_relabelling(oracle_mod):
    """Only global links with the identity relabelling: the target index i
    has P(i >= x) = P(D(1024) >= x + 1024), up to the share 1024 / (n + 1024)
    of draws that wrap modulo n.  With perm (a, b) every target is
    a*i + b mod n of the identity run."""
    n = 1 << 20
    ident = _model(p_zero=0, p_home=0, p_local=0, perm_a=1, perm_b=0)
    perm = _model(p_zero=0, p_home=0, p_local=0)
    us = range(0, n, 97)
    i = np.concatenate([oracle_mod.web_row_links(n, 9, ident, u) for u in us]).astype(np.int64)
    N = len(i)
    wrap = 1024 / (n + 1024)
    for x in (1024, 3072, 31744):
        p = float(_pareto_tail(1024, x + 1024))
        assert abs((i >= x).mean() - p) < 5 * np.sqrt(p * (1 - p) / N) + wrap
    v = np.concatenate([oracle_mod.web_row_links(n, 9, perm, u) for u in us])
    assert len(v) == N
    a, b = perm["perm_a"], perm["perm_b"]
    want = (np.uint64(a) * i.astype(np.uint64) + np.uint64(b)) % np.uint64(n)
    assert np.array_equal(v.astype(np.uint64), want)


def test_web_seeded(oracle_mod):
    a = oracle_mod.web_edges(2000, 1, MODEL)
    b = oracle_mod.web_edges(2000, 1, MODEL)
    c = oracle_mod.web_edges(2000, 2, MODEL)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert len(a[0]) != len(c[0]) or not np.array_equal(a[1], c[1])


def test_web_rows_match_whole_graph(oracle_mod):
    """Rows of CSR(A) and CSR(A^T) regenerated one at a time equal those of
    the graph built from the whole link list."""
    n = 5000
    g = oracle_mod.web_graph(n, 6, MODEL)
    rng = np.random.default_rng(0)
    us = rng.choice(n, 40, replace=False).tolist() + [0, n - 1]
    for u in us:
        assert np.array_equal(oracle_mod.web_out_row(n, 6, MODEL, u),
                              g.col[g.rowptr[u]:g.rowptr[u + 1]]), u
    vs = us + [int(np.argmax(g.indeg))]
    rows = oracle_mod.web_in_rows(n, 6, MODEL, vs)
    for v in vs:
        assert np.array_equal(rows[v], g.colT[g.rowptrT[v]:g.rowptrT[v + 1]]), v


@pytest.mark.parametrize("n", [1 << 16])
def test_web_shape(oracle_mod, n):
    """The stand-in's shape: high mean degree after merging repeats, a share
    of pages without links, most links short, a few very popular pages."""
    g = oracle_mod.web_graph(n, synthetic.WEB_SEED, MODEL)
    assert 30 < g.m / n < 45
    assert abs((g.outdeg == 0).mean() - MODEL["p_zero"] / 65536) < 0.01
    rows = np.repeat(np.arange(n), np.diff(g.rowptr))
    dist = np.abs(rows - g.col)
    dist = np.minimum(dist, n - dist)
    assert (dist < 1024).mean() > 0.3
    assert g.indeg.max() > 100 * g.m / n
