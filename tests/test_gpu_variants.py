"""Every tile-plan variant the autotuner may choose (workgroup or wavefront
tiles, LDS hot slice, degree relabeling) computes the same PageRank up to
floating-point reassociation (the paper's rule that algorithm selection
never changes results, Section III-D), checked against the FP64 oracle."""
import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu

D = 0.85

VARIANTS = [
    dict(kernel=0, lds_entries=2048, lds_rows=1024, long_row=2048, chunk=2048, grid=0, hot=0, relabel=0),
    dict(kernel=0, lds_entries=1024, lds_rows=512, long_row=256, chunk=1024, grid=0, hot=0, relabel=0),
    dict(kernel=0, lds_entries=4096, lds_rows=1024, long_row=512, chunk=4096, grid=3, hot=0, relabel=1),
    dict(kernel=1, lds_entries=512, lds_rows=256, long_row=512, chunk=512, grid=0, hot=0, relabel=0),
    dict(kernel=1, lds_entries=512, lds_rows=256, long_row=512, chunk=512, grid=0, hot=1 << 20, relabel=0),
    dict(kernel=1, lds_entries=512, lds_rows=256, long_row=64, chunk=512, grid=0, hot=1 << 20, relabel=1),
    dict(kernel=1, lds_entries=512, lds_rows=256, long_row=128, chunk=256, grid=5, hot=1000, relabel=1),
    # tiles split into one contiguous range per XCD (grid a multiple of 8;
    # with grid 5 the split is ignored)
    dict(kernel=0, lds_entries=2048, lds_rows=1024, long_row=2048, chunk=2048, grid=16, hot=0, relabel=0,
         xcd_split=1),
    dict(kernel=0, lds_entries=1024, lds_rows=512, long_row=256, chunk=1024, grid=4096, hot=0, relabel=1,
         xcd_split=1),
    dict(kernel=1, lds_entries=512, lds_rows=256, long_row=512, chunk=512, grid=0, hot=1 << 20, relabel=1,
         xcd_split=1),
    dict(kernel=1, lds_entries=512, lds_rows=256, long_row=64, chunk=512, grid=8, hot=0, relabel=0,
         xcd_split=1),
    dict(kernel=1, lds_entries=512, lds_rows=256, long_row=128, chunk=256, grid=5, hot=1000, relabel=1,
         xcd_split=1),
]


def _ids(v):
    return "k%d-e%d-l%d-c%d-g%d-h%d-r%d-x%d" % (v["kernel"], v["lds_entries"], v["long_row"], v["chunk"],
                                              v["grid"], v["hot"], v["relabel"], v.get("xcd_split", 0))


def _run(grb, g, dtype, cfg, **kw):
    from paper_2509_14211_amd import api
    t = grb.builtin("GrB_FP32" if dtype == torch.float32 else "GrB_FP64")
    grb.GrM_Matrix_plan_set(g.AT, t, cfg)
    try:
        x, it, res = api.pagerank(g, dtype, **kw)
    finally:
        grb.GrM_Matrix_plan_set(g.AT, t, None)
    return x.cpu().numpy().astype(np.float64), it, res


@pytest.mark.parametrize("cfg", VARIANTS, ids=_ids)
def test_variant_rmat(nonblocking, oracle_mod, cfg):
    from paper_2509_14211_amd import api
    print("variant", _ids(cfg), flush=True)
    g = api.rmat_graph(12)
    og = oracle_mod.rmat_graph(12)
    x, it, res = _run(nonblocking, g, torch.float64, cfg, tol=1e-10)
    ref = oracle_mod.pagerank(og, D, fixed_iters=it)
    assert np.abs(x - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12
    assert abs(res - ref.resid) <= 4 * np.abs(x - ref.x).sum() + 1e-16
    x, it, res = _run(nonblocking, g, torch.float32, cfg, tol=1e-6)
    ref = oracle_mod.pagerank(og, D, fixed_iters=it)
    assert np.abs(x - ref.x).sum() <= 1e-5
    x, it, _ = _run(nonblocking, g, torch.float64, cfg, tol=1e-9, dangling=0)
    ref = oracle_mod.pagerank(og, D, fixed_iters=it, mode=0)
    assert np.abs(x - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12
    g.free()


@pytest.mark.parametrize("cfg", VARIANTS, ids=_ids)
def test_variant_hub_and_edge_graphs(nonblocking, cfg):
    from paper_2509_14211_amd import api
    m = 20000
    for spec, want in (
        (synthetic.star_in(m), lambda x: (abs(x[0] - (1 + m * D) / (m + 1 + m * D)) < 1e-13 and
                                          np.allclose(x[1:], 1 / (m + 1 + m * D), rtol=1e-12, atol=0))),
        (synthetic.star_both(700), lambda x: abs(x[0] - (1 + D * 700) / (701 * (1 + D))) < 1e-13),
        (synthetic.empty(5), lambda x: np.allclose(x, 0.2, rtol=1e-14, atol=0)),
        (synthetic.cycle(3), lambda x: np.allclose(x, 1 / 3, rtol=1e-14, atol=0)),
    ):
        n, src, dst = spec
        g = api.graph_from_edges(n, src, dst)
        x, _, _ = _run(nonblocking, g, torch.float64, cfg, tol=1e-14, itermax=400)
        assert want(x), _ids(cfg)
        g.free()


def test_variant_x0_with_relabel(nonblocking, oracle_mod):
    from paper_2509_14211_amd import api
    g = api.rmat_graph(11)
    og = oracle_mod.rmat_graph(11)
    x0 = synthetic.random_distribution(g.n, 9)
    cfg = VARIANTS[5]
    t = nonblocking.builtin("GrB_FP64")
    nonblocking.GrM_Matrix_plan_set(g.AT, t, cfg)
    x, it, _ = api.pagerank(g, torch.float64, tol=1e-10, x0=torch.from_numpy(x0))
    nonblocking.GrM_Matrix_plan_set(g.AT, t, None)
    ref = oracle_mod.pagerank(og, D, fixed_iters=it, x0=x0)
    x = x.cpu().numpy()
    assert np.abs(x - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12
    g.free()


def test_plan_config_validation(nonblocking):
    from paper_2509_14211_amd import api
    grb = nonblocking
    g = api.rmat_graph(8)
    t = grb.builtin("GrB_FP32")
    bad = [dict(kernel=4, lds_entries=2048, lds_rows=1024, long_row=2048, chunk=2048),
           dict(kernel=0, lds_entries=3000, lds_rows=1024, long_row=2048, chunk=2048),
           dict(kernel=1, lds_entries=2048, lds_rows=1024, long_row=512, chunk=512),
           dict(kernel=0, lds_entries=2048, lds_rows=1024, long_row=4096, chunk=2048),
           dict(kernel=1, lds_entries=512, lds_rows=256, long_row=512, chunk=1024),
           dict(kernel=1, lds_entries=512, lds_rows=256, long_row=512, chunk=512, xcd_split=2)]
    for cfg in bad:
        with pytest.raises(grb.GrBError) as e:
            grb.GrM_Matrix_plan_set(g.AT, t, cfg)
        assert e.value.info == -3
    got = grb.GrM_Matrix_plan_get(g.AT, t)
    assert got["lds_entries"] in (512, 1024, 2048, 4096)
    g.free()
