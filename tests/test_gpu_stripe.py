"""The stripe-blocked fused pass (plan kernel 2: row stripes with their sums
in LDS, leading column blocks of the gathered vector staged through LDS,
the other entries gathered from memory, 64-bit fixed-point row sums)
computes the Fig. 6 PageRank pass: every configuration is checked against
the FP64 oracle at the same pass count, per vertex as well as in L1, on
graphs that span several stripes and column blocks with ragged tails, on
hub rows, and on the degenerate graphs.  Integer-valued operands make the
fixed-point sums exact, which pins the accumulation bit for bit."""
import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu

D = 0.85
HB = 12288


def stripe_cfg(relabel=1, long_row=1024, hot=0, grid=0, chunk=0, kernel=2):
    return dict(kernel=kernel, lds_entries=0, lds_rows=0, long_row=long_row, chunk=chunk, grid=grid, hot=hot,
                relabel=relabel)


CONFIGS = [
    stripe_cfg(),
    stripe_cfg(relabel=0),
    stripe_cfg(long_row=1),               # every block holding an entry is loaded
    stripe_cfg(long_row=1 << 30),         # no block is loaded: every entry gathered
    stripe_cfg(hot=HB, grid=3),           # one LDS block at most, three workgroups
    stripe_cfg(hot=2 * HB, long_row=64, grid=13),
    stripe_cfg(chunk=1),                  # packed entries read with the nontemporal hint
    # two-phase: the entries outside the LDS blocks are filled block by block
    stripe_cfg(kernel=3),
    stripe_cfg(kernel=3, relabel=0, chunk=1),
    stripe_cfg(kernel=3, long_row=1 << 30),  # no LDS block: every entry filled
    stripe_cfg(kernel=3, hot=HB, grid=3),
]


def _ids(c):
    return "k%d-r%d-l%d-h%d-g%d-c%d" % (c["kernel"], c["relabel"], c["long_row"], c["hot"], c["grid"], c["chunk"])


def _run(grb, g, cfg, dtype=torch.float32, **kw):
    from paper_2509_14211_amd import api
    t = grb.builtin("GrB_FP32" if dtype == torch.float32 else "GrB_FP64")
    grb.GrM_Matrix_plan_set(g.AT, t, cfg)
    try:
        x, it, res = api.pagerank(g, dtype, **kw)
    finally:
        grb.GrM_Matrix_plan_set(g.AT, t, None)
    return x.cpu().numpy().astype(np.float64), it, res


def _check_fp32(x, ref_x):
    err = np.abs(x - ref_x)
    assert err.sum() <= 1e-5, err.sum()
    # per vertex: FP32 rounding of each pass, not a localized error
    bad = err > 1e-4 * np.abs(ref_x) + 1e-9
    assert not bad.any(), (np.flatnonzero(bad)[:10], err[bad][:10], ref_x[bad][:10])


@pytest.mark.parametrize("cfg", CONFIGS, ids=_ids)
@pytest.mark.parametrize("scale", [12, 17])
def test_stripe_rmat_matches_oracle(nonblocking, oracle_mod, cfg, scale):
    from paper_2509_14211_amd import api
    print("stripe", _ids(cfg), "scale", scale, flush=True)
    g = api.rmat_graph(scale)
    og = oracle_mod.rmat_graph(scale)
    for dangling in (1, 0):
        x, it, res = _run(nonblocking, g, cfg, tol=1e-6, dangling=dangling)
        ref = oracle_mod.pagerank(og, D, fixed_iters=it, mode=dangling)
        _check_fp32(x, ref.x)
        assert abs(res - ref.resid) <= 4 * np.abs(x - ref.x).sum() + 1e-9
        if dangling == 1:
            assert abs(x.sum() - 1.0) <= 1e-5
    # free-running to a tight tolerance, against the fixed point
    x, it, res = _run(nonblocking, g, cfg, tol=1e-7, itermax=300)
    ref = oracle_mod.pagerank(og, D, tol=1e-13, itermax=1000)
    assert np.abs(x - ref.x).sum() <= D / (1 - D) * 1e-7 + 2e-6
    g.free()


def test_stripe_many_blocks_and_cold_entries(nonblocking, oracle_mod):
    """Scale 19: 524,288 columns = 42.7 blocks of 12,288, so with every
    block eligible a stripe loads up to 43 of them, and with at most 32
    (hot cap) it gathers the rest; at least 66 stripes of at most 8064
    rows each."""
    from paper_2509_14211_amd import api
    g = api.rmat_graph(19)
    og = oracle_mod.rmat_graph(19)
    for cfg in (stripe_cfg(long_row=1), stripe_cfg(relabel=0, long_row=1), stripe_cfg(long_row=1, hot=32 * HB),
                stripe_cfg(kernel=3, long_row=1), stripe_cfg(kernel=3, relabel=0, long_row=2048)):
        x, it, _ = _run(nonblocking, g, cfg, tol=1e-6)
        ref = oracle_mod.pagerank(og, D, fixed_iters=it)
        _check_fp32(x, ref.x)
    g.free()


def test_stripe_is_deterministic(nonblocking):
    from paper_2509_14211_amd import api
    g = api.rmat_graph(16)
    a, ita, ra = _run(nonblocking, g, stripe_cfg(), tol=1e-7)
    b, itb, rb = _run(nonblocking, g, stripe_cfg(), tol=1e-7)
    assert ita == itb and ra == rb and np.array_equal(a, b)
    g.free()


@pytest.mark.parametrize("cfg", [stripe_cfg(), stripe_cfg(long_row=1 << 30), stripe_cfg(grid=2)], ids=_ids)
def test_stripe_hub_and_edge_graphs(nonblocking, cfg):
    from paper_2509_14211_amd import api
    m = 40000
    for spec, want in (
        # one row of 40000 entries: whole wavefronts of one row
        (synthetic.star_in(m), lambda x: (abs(x[0] - (1 + m * D) / (m + 1 + m * D)) < 1e-6 and
                                          np.allclose(x[1:], 1 / (m + 1 + m * D), rtol=1e-5, atol=0))),
        (synthetic.star_out(m), lambda x: (abs(x[0] - 1 / (m + 1 + D)) < 1e-6 and
                                           np.allclose(x[1:], (m + D) / (m * (m + 1 + D)), rtol=1e-5, atol=0))),
        (synthetic.star_both(700), lambda x: abs(x[0] - (1 + D * 700) / (701 * (1 + D))) < 1e-6),
        (synthetic.empty(5), lambda x: np.allclose(x, 0.2, rtol=1e-6, atol=0)),
        (synthetic.cycle(3), lambda x: np.allclose(x, 1 / 3, rtol=1e-6, atol=0)),
        (synthetic.cycle(20000), lambda x: np.allclose(x, 1 / 20000, rtol=1e-5, atol=0)),
    ):
        n, src, dst = spec
        g = api.graph_from_edges(n, src, dst)
        x, _, _ = _run(nonblocking, g, cfg, tol=1e-9, itermax=400)
        assert want(x), _ids(cfg)
        g.free()


@pytest.mark.parametrize("scale", [9, 17, 21])
def test_stripe_mxv_exact_on_integers(blocking, scale):
    """Blocking-mode GrB_mxv on the stripe plan: with integer-valued FP32
    operands (|sums| < 2^24) every fixed-point term and row sum is exact, so
    the product equals the exact one bit for bit, signs included."""
    from paper_2509_14211_amd import api
    grb = blocking
    g = api.rmat_graph(scale)
    rowptr, col = api.csr_of(g.AT)
    rp = rowptr.cpu().numpy().astype(np.int64)
    cl = col.cpu().numpy().astype(np.int64)
    rng = np.random.default_rng(5)
    u = rng.integers(-8, 9, size=g.n).astype(np.float32)
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    exact = np.zeros(g.n, np.float64)
    np.add.at(exact, rows, u[cl].astype(np.float64))
    t = grb.builtin("GrB_FP32")
    for cfg in (stripe_cfg(relabel=0), stripe_cfg(relabel=0, long_row=1 << 30), stripe_cfg(relabel=0, grid=5),
                stripe_cfg(relabel=0, kernel=3), stripe_cfg(relabel=0, kernel=3, long_row=1 << 30)):
        grb.GrM_Matrix_plan_set(g.AT, t, cfg)
        uv = api.vector_from_tensor(torch.from_numpy(u).cuda())
        w = grb.GrB_Vector_new(t, g.n)
        grb.GrB_mxv(w, None, None, grb.builtin("GrB_PLUS_TIMES_SEMIRING_FP32"), g.AT, uv)
        got = api.tensor_from_vector(w, torch.float32).cpu().numpy().astype(np.float64)
        grb.GrM_Matrix_plan_set(g.AT, t, None)
        for h in (uv, w):
            grb.GrB_Vector_free(h)
        assert np.array_equal(got, exact), (_ids(cfg), np.flatnonzero(got != exact)[:10])
    g.free()


def test_stripe_nan_start_is_an_execution_error(nonblocking):
    from paper_2509_14211_amd import api
    grb = nonblocking
    g = api.rmat_graph(12)
    x0 = torch.full((g.n,), 1.0 / g.n, dtype=torch.float32)
    x0[17] = float("nan")
    t = grb.builtin("GrB_FP32")
    grb.GrM_Matrix_plan_set(g.AT, t, stripe_cfg())
    try:
        with pytest.raises(grb.GrBError) as e:
            api.pagerank(g, torch.float32, tol=1e-6, x0=x0)
        assert e.value.info == -101
    finally:
        grb.GrM_Matrix_plan_set(g.AT, t, None)
    # the library stays usable: the next solve on the same plan is exact
    x, it, _ = _run(grb, g, stripe_cfg(), tol=1e-6)
    assert np.isfinite(x).all() and abs(x.sum() - 1.0) < 1e-5
    g.free()


def test_stripe_plan_only_for_fp32(nonblocking):
    from paper_2509_14211_amd import api
    grb = nonblocking
    g = api.rmat_graph(8)
    for kernel in (2, 3):
        with pytest.raises(grb.GrBError) as e:
            grb.GrM_Matrix_plan_set(g.AT, grb.builtin("GrB_FP64"), stripe_cfg(kernel=kernel))
        assert e.value.info == -3
    g.free()


def test_two_phase_stripe_is_deterministic_and_matches_gathered(nonblocking):
    """The two-phase plan regroups entries with atomics (their order inside
    a block group varies from build to build), yet its fixed-point sums are
    exact: two builds give the same bits, and integer products equal the
    gathered plan's."""
    from paper_2509_14211_amd import api
    g = api.rmat_graph(16)
    a, ita, ra = _run(nonblocking, g, stripe_cfg(kernel=3), tol=1e-7)
    g.free()
    g = api.rmat_graph(16)
    b, itb, rb = _run(nonblocking, g, stripe_cfg(kernel=3), tol=1e-7)
    c, itc, rc = _run(nonblocking, g, stripe_cfg(kernel=2), tol=1e-7)
    assert ita == itb and ra == rb and np.array_equal(a, b)
    assert itc == ita and np.array_equal(a, c)
    g.free()


def _mxv_fp32(grb, A, u):
    from paper_2509_14211_amd import api
    t = grb.builtin("GrB_FP32")
    uv = api.vector_from_tensor(u)
    w = grb.GrB_Vector_new(t, grb.GrB_Matrix_nrows(A))
    try:
        grb.GrB_mxv(w, None, None, grb.builtin("GrB_PLUS_TIMES_SEMIRING_FP32"), A, uv)
        return api.tensor_from_vector(w, torch.float32)
    finally:
        grb.GrB_Vector_free(uv)
        grb.GrB_Vector_free(w)


def _exact(rowptr, col, u):
    rows = torch.repeat_interleave(torch.arange(rowptr.numel() - 1, device="cuda"),
                                   (rowptr[1:] - rowptr[:-1]).long())
    return torch.zeros(rowptr.numel() - 1, dtype=torch.float64, device="cuda").index_add_(
        0, rows, u[col.long()].double())


def test_stripe_loads_the_dense_blocks_of_a_banded_graph(nonblocking, oracle_mod):
    """Links only to nearby vertices: each stripe's entries sit in the one
    or two column blocks around its own rows, not in the leading blocks.
    The layout picks those blocks (so most entries read LDS) and the
    results are exact on integers and match the oracle per vertex."""
    from paper_2509_14211_amd import api
    n = 150000
    i = np.repeat(np.arange(n), 6)
    d = np.tile(np.array([-3000, -700, -1, 1, 500, 2500]), n)
    src = i.astype(np.uint32)
    dst = ((i + d) % n).astype(np.uint32)
    g = api.graph_from_edges(n, src, dst)
    og = oracle_mod.graph_from_edges(n, src, dst)
    grb = nonblocking
    t = grb.builtin("GrB_FP32")
    for cfg in (stripe_cfg(relabel=0, long_row=256), stripe_cfg(relabel=0, long_row=256, kernel=3)):
        # integer mxv, bit for bit
        grb.GrM_set_mode(grb.GrB_BLOCKING)
        grb.GrM_Matrix_plan_set(g.AT, t, cfg)
        try:
            rp, cl = api.csr_of(g.AT)
            gen = torch.Generator(device="cuda")
            gen.manual_seed(3)
            u = torch.randint(-8, 9, (n,), device="cuda", generator=gen).float()
            got = _mxv_fp32(grb, g.AT, u).double()
            assert torch.equal(got, _exact(rp, cl, u)), _ids(cfg)
        finally:
            grb.GrM_Matrix_plan_set(g.AT, t, None)
            grb.GrM_set_mode(grb.GrB_NONBLOCKING)
        x, it, _ = _run(nonblocking, g, cfg, tol=1e-7)
        ref = oracle_mod.pagerank(og, D, fixed_iters=it)
        _check_fp32(x, ref.x)
    g.free()


def test_stripe_with_more_column_blocks_than_the_layout_tells_apart(blocking):
    """205M columns (16,685 blocks of 12,288, more than the 16,384 the
    layout counts one by one): blocks from 16,383 on share one bin that is
    never loaded, so their entries are gathered; a dense low block is still
    loaded.  Integer operands, exact."""
    from paper_2509_14211_amd import api
    grb = blocking
    nrows, ncols = 16128, 205_000_000
    hb = 12288
    gen = torch.Generator(device="cuda")
    gen.manual_seed(9)
    per = 48
    # per row: 24 distinct columns in block 3, 12 in blocks >= 16383, 12 anywhere
    lo = 3 * hb + torch.stack([torch.randperm(hb, device="cuda", generator=gen)[:24] for _ in range(4)])
    lo = lo[torch.arange(nrows, device="cuda") % 4]
    hi = 16383 * hb + torch.randint(0, ncols - 16383 * hb, (nrows, 12), device="cuda", generator=gen)
    anyc = torch.randint(0, ncols, (nrows, 12), device="cuda", generator=gen)
    cols = torch.cat([lo, hi, anyc], dim=1)
    cols, _ = torch.sort(cols, dim=1)
    keep = torch.ones_like(cols, dtype=torch.bool)
    keep[:, 1:] = cols[:, 1:] != cols[:, :-1]
    counts = keep.sum(dim=1)
    rowptr = torch.zeros(nrows + 1, dtype=torch.int32, device="cuda")
    rowptr[1:] = torch.cumsum(counts, 0).int()
    col = cols[keep].int().contiguous()
    assert col.numel() == int(rowptr[-1]) and per * nrows >= col.numel()
    A = grb.GrB_Matrix_new(grb.builtin("GrB_FP32"), nrows, ncols)
    t = grb.builtin("GrB_FP32")
    try:
        grb.GrM_Matrix_import_CSR(A, rowptr, col, col.numel())
        u = torch.randint(-8, 9, (ncols,), device="cuda", generator=gen).float()
        want = _exact(rowptr, col, u)
        for cfg in (stripe_cfg(relabel=0, long_row=1000), stripe_cfg(relabel=0, long_row=1),
                    stripe_cfg(relabel=0, long_row=1000, kernel=3)):
            grb.GrM_Matrix_plan_set(A, t, cfg)
            got = _mxv_fp32(grb, A, u).double()
            grb.GrM_Matrix_plan_set(A, t, None)
            assert torch.equal(got, want), cfg
    finally:
        grb.GrB_Matrix_free(A)
