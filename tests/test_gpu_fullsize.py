"""Parity at the workload sizes, in the launch configuration the benchmark
times (autotuned plan): the R-MAT scale-22 and scale-25 solves against the
full FP64 oracle (L1 and per vertex), the stripe-blocked plan forced at
scale 22, every column of the 64-set batched PPR and every set of a
128-set PPR stream, all 256 graphs of the many-graph workload, and the
warm-start network on sampled vertices of the scale-22 graph."""
import os

import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu

D = 0.85


def _threads():
    return min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def g22(gpu, oracle_mod):
    from paper_2509_14211_amd import api
    print("scale-22 graph, GPU and oracle", flush=True)
    oracle_mod.set_threads(_threads())
    g = api.rmat_graph(22)
    for t in ("GrB_FP32", "GrB_FP64"):
        gpu.GrM_autotune_pagerank(g.AT, g.outdeg, gpu.builtin(t), None)
    og = oracle_mod.rmat_graph(22)
    yield g, og
    g.free()


def test_scale22_graph_is_bit_exact(gpu, g22):
    from paper_2509_14211_amd import api
    g, og = g22
    assert g.m == og.m
    rp, col = api.csr_of(g.AT)
    assert np.array_equal(rp.cpu().numpy(), og.rowptrT)
    assert np.array_equal(col.cpu().numpy(), og.colT)
    deg = api.tensor_from_vector(g.outdeg, torch.int32).cpu().numpy()
    assert np.array_equal(deg, og.outdeg)


def test_scale22_fp32_fused_matches_oracle(gpu, oracle_mod, g22):
    """The headline solve: FP32 ranks with FP64 reductions to L1 1e-6."""
    from paper_2509_14211_amd import api
    g, og = g22
    x, it, res = api.pagerank(g, torch.float32, D, 1e-6)
    x = x.cpu().numpy().astype(np.float64)
    ref = oracle_mod.pagerank(og, D, fixed_iters=it)
    err = np.abs(x - ref.x).sum()
    print("scale 22 fp32: %d passes, L1 error %.3e" % (it, err), flush=True)
    assert err <= 1e-5
    _per_vertex(x, ref.x)
    assert res <= 1e-6 and abs(res - ref.resid) <= 4 * err + 1e-7
    assert abs(x.sum() - 1.0) <= 1e-5
    free = oracle_mod.pagerank(og, D, tol=1e-6)
    assert abs(it - free.iters) <= 1


def _per_vertex(x, ref_x):
    """No localized error hides under the L1 bound: every vertex within
    1e-4 of its own rank (plus 1e-9)."""
    e = np.abs(x - ref_x)
    bad = e > 1e-4 * np.abs(ref_x) + 1e-9
    assert not bad.any(), (np.flatnonzero(bad)[:10], e[bad][:10])


@pytest.mark.parametrize("kernel,relabel", [(2, 1), (2, 0), (3, 1), (3, 0)])
def test_scale22_stripe_plan_matches_oracle(gpu, oracle_mod, g22, kernel, relabel):
    """The stripe-blocked pass (row sums in LDS, dense column blocks in LDS,
    64-bit fixed-point sums), gathered (kernel 2) or two-phase (kernel 3),
    at the headline size."""
    from paper_2509_14211_amd import api
    g, og = g22
    t = gpu.builtin("GrB_FP32")
    saved = gpu.GrM_Matrix_plan_get(g.AT, t)
    gpu.GrM_Matrix_plan_set(g.AT, t, dict(kernel=kernel, lds_entries=0, lds_rows=0, long_row=1024, chunk=0,
                                          grid=0, hot=0, relabel=relabel))
    try:
        x, it, res = api.pagerank(g, torch.float32, D, 1e-6)
    finally:
        gpu.GrM_Matrix_plan_set(g.AT, t, saved)
    x = x.cpu().numpy().astype(np.float64)
    ref = oracle_mod.pagerank(og, D, fixed_iters=it)
    err = np.abs(x - ref.x).sum()
    print("scale 22 stripe kernel %d relabel %d: %d passes, L1 error %.3e" % (kernel, relabel, it, err),
          flush=True)
    assert err <= 1e-5
    _per_vertex(x, ref.x)
    assert res <= 1e-6 and abs(res - ref.resid) <= 4 * err + 1e-7


def test_scale22_fp64_fused_matches_oracle(gpu, oracle_mod, g22):
    from paper_2509_14211_amd import api
    g, og = g22
    x, it, res = api.pagerank(g, torch.float64, D, 1e-9)
    x = x.cpu().numpy()
    ref = oracle_mod.pagerank(og, D, fixed_iters=it)
    assert np.abs(x - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12
    assert abs(res - ref.resid) <= 4 * np.abs(x - ref.x).sum() + 1e-16


def test_scale22_ppr_batch_all_columns(gpu, oracle_mod, g22):
    """64 seed sets (sizes 1..16, seed 7) as one SpMM solve to 1e-6: every
    column against the single-vector oracle after its own pass count (a
    column stops where its residual first reaches the tolerance), in L1 and
    per vertex."""
    g, og = g22
    sets = [s.tolist() for s in synthetic.ppr_seed_sets(g.n, 64, seed=7)]
    X = torch.empty(g.n * 64, dtype=torch.float32, device="cuda")
    it, col_it, col_res = gpu.GrM_ppr_batch(X, gpu.builtin("GrB_FP32"), sets, g.AT, g.outdeg, D, 1e-6, 1000)
    X = X.reshape(g.n, 64).cpu().numpy().astype(np.float64)
    assert col_res.max() <= 1e-6
    assert np.all(np.abs(X.sum(axis=0) - 1.0) <= 1e-5)
    assert it == col_it.max() and col_it.min() >= 1
    for q in range(64):
        print("ppr batch column %d (%d passes)" % (q, col_it[q]), flush=True)
        ref = oracle_mod.ppr(og, sets[q], D, fixed_iters=int(col_it[q]))
        assert np.abs(X[:, q] - ref.x).sum() <= 1e-5, q
        _per_vertex(X[:, q], ref.x)


def test_scale22_ppr_stream_128_sets(gpu, oracle_mod, g22):
    """128 seed sets streamed through 64 columns (converged columns retire
    and restart with the next set): every set against the single-vector
    oracle after the passes it ran, in L1 and per vertex."""
    g, og = g22
    sets = [s.tolist() for s in synthetic.ppr_seed_sets(g.n, 128, seed=8)]
    X = torch.empty(g.n * 128, dtype=torch.float32, device="cuda")
    first, ran, res = gpu.GrM_ppr_stream(X, gpu.builtin("GrB_FP32"), sets, g.AT, g.outdeg, D, 1e-6, 1000)
    X = X.reshape(128, g.n).cpu().numpy().astype(np.float64)
    assert res.max() <= 1e-6
    for q in range(128):
        print("ppr stream set %d (%d passes)" % (q, int(ran[q])), flush=True)
        ref = oracle_mod.ppr(og, sets[q], D, fixed_iters=int(ran[q]))
        assert np.abs(X[q] - ref.x).sum() <= 1e-5, q
        _per_vertex(X[q], ref.x)


def test_scale22_warm_start_sampled_vertices(gpu, oracle_mod, g22):
    """Walk counts of the whole graph bit-exact; z of sampled vertices
    (small two-hop in-neighbourhoods) against the oracle's one-by-one
    evaluation, FP32 activations."""
    from oracle import gnn
    from paper_2509_14211_amd import api
    g, og = g22
    seeds = [int(v) for v in synthetic.ppr_seed_sets(g.n, 1, seed=77)[0]]
    rng = np.random.default_rng(3)
    theta = (gnn.init_params(3) + 0.05 * rng.normal(size=gnn.NPARAMS)).astype(np.float32)
    W = 1 << 14
    net = gpu.GrM_GNN_new(gpu.builtin("GrB_FP32"), 0)
    try:
        gpu.GrM_GNN_set_params(net, theta)
        gpu.GrM_gnn_features(net, g.A, g.AT, seeds, W, D, 2024)
        gpu.GrM_gnn_forward(net, g.A, g.AT)
        p, c = gpu.GrM_GNN_buffer(net, "counts")
        counts = api.device_copy(p, c, torch.int32).cpu().numpy().reshape(gnn.STEPS, g.n)
        assert np.array_equal(counts, gnn.walk_counts(og, seeds, W, D, 2024))
        p, c = gpu.GrM_GNN_buffer(net, "z")
        z = api.device_copy(p, c, torch.float32).cpu().numpy().astype(np.float64)
    finally:
        gpu.GrM_GNN_free(net)
    X = gnn.features(og, seeds, W, D, 2024)
    indeg = np.diff(og.rowptrT)
    cand = [v for v in rng.choice(g.n, 4000, replace=False)
            if indeg[v] <= 64 and indeg[og.colT[og.rowptrT[v]:og.rowptrT[v + 1]]].sum() <= 4000]
    vs = [int(v) for v in cand[:48]] + [int(s) for s in seeds]
    want = gnn.z_at(og, theta.astype(np.float64), lambda u: X[u], vs)
    assert np.abs(z[vs] - want).max() <= 1e-5 * max(np.abs(want).max(), 1.0)


def test_many_graphs_full_workload(gpu, oracle_mod):
    """All 256 graphs (scales 10..16) in one persistent launch, each against
    the oracle at its own pass count."""
    from paper_2509_14211_amd import api
    specs = synthetic.many_graph_specs(256)
    gs = [api.rmat_graph(s, 16, seed) for s, seed in specs]
    mg = gpu.GrM_Multigraph_new([x.AT for x in gs])
    try:
        off = gpu.GrM_Multigraph_offsets(mg, len(gs))
        X = torch.empty(int(off[-1]), dtype=torch.float32, device="cuda")
        its, res = gpu.GrM_pagerank_many(X, gpu.builtin("GrB_FP32"), mg, len(gs), D, 1e-6, 1000)
        x = X.cpu().numpy().astype(np.float64)
        assert np.all(res <= 1e-6)
        for i, (s, seed) in enumerate(specs):
            og = oracle_mod.rmat_graph(s, 16, seed)
            ref = oracle_mod.pagerank(og, D, fixed_iters=int(its[i]))
            assert np.abs(x[off[i]:off[i + 1]] - ref.x).sum() <= 1e-5, (i, s)
    finally:
        gpu.GrM_Multigraph_free(mg)
        for x_ in gs:
            x_.free()


def test_scale25_stripe_mxv_exact_on_integers(gpu):
    """The stripe layout at scale 25 (about 4,200 stripes of up to 8064
    rows, 2,731 column blocks): with integer-valued FP32 operands every
    fixed-point term and row sum is exact, so GrB_mxv on the stripe plan
    equals the exact product bit for bit -- each entry is placed exactly
    once, in its own row, with and without the degree renumbering."""
    from paper_2509_14211_amd import api
    print("scale-25 graph on the GPU (integer mxv)", flush=True)
    g = api.rmat_graph(25)
    t = gpu.builtin("GrB_FP32")
    try:
        rp, col = api.csr_of(g.AT)
        rows = torch.repeat_interleave(torch.arange(g.n, device="cuda"), (rp[1:] - rp[:-1]).long())
        gen = torch.Generator(device="cuda")
        gen.manual_seed(5)
        u = torch.randint(-8, 9, (g.n,), device="cuda", generator=gen).float()
        exact = torch.zeros(g.n, dtype=torch.float64, device="cuda").index_add_(0, rows, u[col.long()].double())
        del rows, rp, col
        gpu.GrM_set_mode(gpu.GrB_BLOCKING)
        for kernel, relabel in ((2, 0), (2, 1), (3, 0), (3, 1)):
            gpu.GrM_Matrix_plan_set(g.AT, t, dict(kernel=kernel, lds_entries=0, lds_rows=0, long_row=1024,
                                                  chunk=0, grid=0, hot=0, relabel=relabel))
            uv = api.vector_from_tensor(u)
            w = gpu.GrB_Vector_new(t, g.n)
            try:
                gpu.GrB_mxv(w, None, None, gpu.builtin("GrB_PLUS_TIMES_SEMIRING_FP32"), g.AT, uv)
                got = api.tensor_from_vector(w, torch.float32).double()
            finally:
                gpu.GrB_Vector_free(uv)
                gpu.GrB_Vector_free(w)
                gpu.GrM_Matrix_plan_set(g.AT, t, None)
            bad = (got != exact).nonzero().flatten()
            print("kernel %d relabel %d: %d rows differ" % (kernel, relabel, bad.numel()), flush=True)
            assert bad.numel() == 0, (kernel, relabel, bad[:10].tolist())
    finally:
        gpu.GrM_set_mode(gpu.GrB_NONBLOCKING)
        g.free()


def test_scale25_fp32_fused_matches_oracle(gpu, oracle_mod):
    """The HBM-bound size: graph bit-exact and the FP32 solve within 1e-5 L1
    of the full FP64 oracle (about a minute of oracle work)."""
    from paper_2509_14211_amd import api
    oracle_mod.set_threads(_threads())
    print("scale-25 graph on the GPU", flush=True)
    g = api.rmat_graph(25)
    try:
        gpu.GrM_autotune_pagerank(g.AT, g.outdeg, gpu.builtin("GrB_FP32"), None)
        x, it, res = api.pagerank(g, torch.float32, D, 1e-6)
        x = x.cpu().numpy().astype(np.float64)
        rp, col = api.csr_of(g.AT)
        rp = rp.cpu().numpy()
        col = col.cpu().numpy()
        print("scale-25 graph in the oracle", flush=True)
        og = oracle_mod.rmat_graph(25)
        assert g.m == og.m
        assert np.array_equal(rp, og.rowptrT) and np.array_equal(col, og.colT)
        del rp, col
        ref = oracle_mod.pagerank(og, D, fixed_iters=it)
        err = np.abs(x - ref.x).sum()
        print("scale 25 fp32: %d passes, L1 error %.3e" % (it, err), flush=True)
        assert err <= 1e-5 and res <= 1e-6
        _per_vertex(x, ref.x)
        assert abs(x.sum() - 1.0) <= 1e-5
    finally:
        g.free()


def test_scale23_fp64_batch_takes_the_wide_kernel(gpu, oracle_mod):
    """64 FP64 columns on R-MAT scale 23: each n x k operand is 4.3 GB, past
    what 32-bit buffer offsets address, so the pass runs the 64-bit
    addressed kernel.  Sampled columns against the oracle at the same pass
    count (relative L1 1e-12), every column's mass 1."""
    from paper_2509_14211_amd import api
    oracle_mod.set_threads(_threads())
    print("scale-23 graph on the GPU", flush=True)
    g = api.rmat_graph(23)
    try:
        assert g.n * 64 * 8 > 0xFFFFFF00
        sets = [s.tolist() for s in synthetic.ppr_seed_sets(g.n, 64, seed=23)]
        X = torch.empty(g.n * 64, dtype=torch.float64, device="cuda")
        it, col_it, col_res = gpu.GrM_ppr_batch(X, gpu.builtin("GrB_FP64"), sets, g.AT, g.outdeg, D, 1e-9, 200)
        print("scale 23 fp64 batch: %d passes" % it, flush=True)
        X = X.reshape(g.n, 64)
        sums = X.sum(dim=0).cpu().numpy()
        assert np.all(np.abs(sums - 1.0) <= 1e-9)
        assert col_res.max() <= 1e-9
        cols = [0, 31, 63]
        Xs = X[:, cols].cpu().numpy()
        del X
        print("scale-23 graph in the oracle", flush=True)
        og = oracle_mod.rmat_graph(23)
        for j, q in enumerate(cols):
            ref = oracle_mod.ppr(og, sets[q], D, fixed_iters=int(col_it[q]))
            assert np.abs(Xs[:, j] - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12, q
    finally:
        g.free()
