"""The web-shaped stand-in for the paper's crawl (Section IV) on the GPU:
the generator and graph build bit-exact against the oracle, PageRank in the
paper's dangling-drop mode against the FP64 oracle, and -- at the full
50.6M-vertex size, in the benchmark's autotuned launch configuration --
sampled rows of A and A^T bit-exact plus a one-pass check of the ranks on
sampled vertices."""
import os

import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu

MODEL = synthetic.WEB_MODEL
D = synthetic.DAMPING


def _np(t):
    return t.cpu().numpy()


@pytest.mark.parametrize("n,seed", [(1, 1), (1000, 2), (65536, 3), (100003, 4)])
def test_web_edges_bitwise(gpu, oracle_mod, n, seed):
    from paper_2509_14211_amd import api
    print("web edges n", n, flush=True)
    src, dst = api.web_device_edges(n, seed, MODEL)
    osrc, odst = oracle_mod.web_edges(n, seed, MODEL)
    assert src.numel() == len(osrc)
    assert np.array_equal(_np(src).view(np.uint32), osrc)
    assert np.array_equal(_np(dst).view(np.uint32), odst)


def test_web_degenerate_and_invalid_models(gpu):
    from paper_2509_14211_amd import api, grb
    none = dict(MODEL, p_zero=65536, p_home=0, p_local=0)
    assert grb.GrM_web_edges(None, None, 0, 1000, 1, none) == 0
    g = api.web_graph(1000, 1, none)
    assert g.m == 0
    g.free()
    for bad in (dict(MODEL, kmin=0), dict(MODEL, kmax=5000), dict(MODEL, kmin=9, kmax=8),
                dict(MODEL, p_home=60000), dict(MODEL, hub=0), dict(MODEL, local_min=4096),
                dict(MODEL, perm_a=2)):
        with pytest.raises(grb.GrBError) as e:
            grb.GrM_web_edges(None, None, 0, 1 << 16, 1, bad)
        assert e.value.info == grb.GrB_INVALID_VALUE, bad
    with pytest.raises(grb.GrBError) as e:
        grb.GrM_web_edges(None, None, 0, 0, 1, MODEL)
    assert e.value.info == grb.GrB_INVALID_VALUE
    m = grb.GrM_web_edges(None, None, 0, 5000, 1, MODEL)
    src = torch.empty(m, dtype=torch.int32, device="cuda")
    with pytest.raises(grb.GrBError) as e:
        grb.GrM_web_edges(src, src, m - 1, 5000, 1, MODEL)
    assert e.value.info == grb.GrB_INSUFFICIENT_SPACE


@pytest.fixture(scope="module")
def web_small(gpu, oracle_mod):
    from paper_2509_14211_amd import api
    n = 200003
    g = api.web_graph(n, 7, MODEL)
    og = oracle_mod.web_graph(n, 7, MODEL)
    yield g, og
    g.free()


def test_web_graph_bitwise(gpu, web_small):
    from paper_2509_14211_amd import api
    g, og = web_small
    assert g.m == og.m
    for A, rp0, col0 in ((g.A, og.rowptr, og.col), (g.AT, og.rowptrT, og.colT)):
        rp, col = api.csr_of(A)
        assert np.array_equal(_np(rp), rp0) and np.array_equal(_np(col), col0)
    assert np.array_equal(_np(api.tensor_from_vector(g.outdeg, torch.int32)), og.outdeg)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("mode", ["drop", "uniform"])
def test_web_pagerank_matches_oracle(gpu, oracle_mod, web_small, dtype, mode):
    """FP32 within 1e-5 L1 and FP64 within 1e-12 relative L1 of the FP64
    oracle at the same number of passes, both dangling modes, autotuned
    (degree-relabelled) plan."""
    from paper_2509_14211_amd import api
    g, og = web_small
    dang = gpu.GrM_DANGLING_DROP if mode == "drop" else gpu.GrM_DANGLING_UNIFORM
    gpu.GrM_autotune_pagerank(g.AT, g.outdeg, api.dtype_code(dtype), None)
    tol = synthetic.WEB_TOL if dtype == torch.float32 else 1e-10
    x, it, res = api.pagerank(g, dtype, D, tol, synthetic.WEB_ITERMAX, dang)
    x = _np(x).astype(np.float64)
    omode = oracle_mod.DROP if mode == "drop" else oracle_mod.UNIFORM
    ref = oracle_mod.pagerank(og, D, mode=omode, fixed_iters=it)
    err = np.abs(x - ref.x).sum()
    print("web n=%d %s %s: %d passes, L1 error %.3e" % (g.n, dtype, mode, it, err), flush=True)
    if dtype == torch.float32:
        assert err <= 1e-5
    else:
        assert err / np.abs(ref.x).sum() <= 1e-12
    assert res <= tol
    free = oracle_mod.pagerank(og, D, tol=tol, itermax=synthetic.WEB_ITERMAX, mode=omode)
    assert abs(it - free.iters) <= 1
    if mode == "drop":
        assert x.sum() < 1.0  # the dangling pages' mass is not returned
    else:
        assert abs(x.sum() - 1.0) <= 1e-5


def _threads():
    return min(16, os.cpu_count() or 1)


def test_web_fullsize_sampled(gpu, oracle_mod):
    """The 50.6M-vertex crawl stand-in: link count, sampled rows of A and
    A^T bit-exact against the oracle's one-row generator, then the FP32
    drop-mode solve in the autotuned plan: residual at tolerance and one
    pass (x_k -> x_k+1) recomputed in FP64 on sampled vertices from the
    oracle's rows."""
    from paper_2509_14211_amd import api
    n, seed = synthetic.WEB_N, synthetic.WEB_SEED
    oracle_mod.set_threads(_threads())
    print("web full size: generating on the GPU", flush=True)
    g = api.web_graph(n, seed, MODEL)
    try:
        assert gpu.GrM_web_edges(None, None, 0, n, seed, MODEL) == int(oracle_mod.web_degrees(n, seed, MODEL).sum())
        rng = np.random.default_rng(11)
        rp, col = api.csr_of(g.A)
        rp = _np(rp)
        us = rng.choice(n, 48, replace=False).tolist() + [0, n - 1, int(np.argmax(np.diff(rp)))]
        print("web full size: rows of A", flush=True)
        for u in us:
            want = oracle_mod.web_out_row(n, seed, MODEL, u)
            got = _np(col[int(rp[u]):int(rp[u + 1])])
            assert np.array_equal(got, want), u
        del col
        rpT, colT = api.csr_of(g.AT)
        rpT = _np(rpT)
        indeg = np.diff(rpT)
        vs = rng.choice(n, 40, replace=False).tolist()
        big = np.argsort(indeg)[-200:]
        vs += [int(v) for v in big[indeg[big] <= 200000][-3:]]
        print("web full size: rows of A^T", flush=True)
        rows = oracle_mod.web_in_rows(n, seed, MODEL, vs)
        for v in vs:
            assert np.array_equal(_np(colT[int(rpT[v]):int(rpT[v + 1])]), rows[v]), v
        del colT
        print("web full size: autotune and solve", flush=True)
        gpu.GrM_autotune_pagerank(g.AT, g.outdeg, gpu.builtin("GrB_FP32"), None)
        x, it, res = api.pagerank(g, torch.float32, D, synthetic.WEB_TOL, synthetic.WEB_ITERMAX,
                                  gpu.GrM_DANGLING_DROP)
        assert res <= synthetic.WEB_TOL and 0.0 < float(x.sum()) < 1.0
        k = 3
        xk, _, _ = api.pagerank(g, torch.float32, D, 0.0, k, gpu.GrM_DANGLING_DROP)
        xk1, _, _ = api.pagerank(g, torch.float32, D, 0.0, k + 1, gpu.GrM_DANGLING_DROP)
        xk = _np(xk).astype(np.float64)
        xk1 = _np(xk1).astype(np.float64)
        outdeg = _np(api.tensor_from_vector(g.outdeg, torch.int32)).astype(np.float64)
        for v in vs:
            src = rows[v]
            for j in src[:8]:
                assert len(oracle_mod.web_out_row(n, seed, MODEL, int(j))) == outdeg[j]
            want = (1.0 - D) / n + D * np.sum(xk[src] / outdeg[src])
            assert abs(xk1[v] - want) <= 1e-5 * want, v
    finally:
        g.free()
