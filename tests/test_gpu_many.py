"""Many independent graphs in one persistent, graph-captured launch: every
graph's ranks against the FP64 oracle at that graph's own pass count, with
and without teams of workgroups per graph, and replays of the captured
launch reproduce the first run bit for bit."""
import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu

D = 0.85


def _graphs(oracle_mod):
    from paper_2509_14211_amd import api
    specs = []
    for scale in range(3, 13):
        src, dst = oracle_mod.rmat_edges(scale, 16, 500 + scale)
        specs.append((1 << scale, src, dst))
    specs += [synthetic.star_in(5000), synthetic.star_both(900), synthetic.empty(7), synthetic.cycle(5),
              synthetic.path2(), synthetic.empty(1), synthetic.complete(40)]
    gs, ogs = [], []
    for n, src, dst in specs:
        gs.append(api.graph_from_edges(n, src, dst))
        ogs.append(oracle_mod.graph_from_edges(n, src, dst))
    return gs, ogs


@pytest.mark.parametrize("team", [8, 1])
@pytest.mark.parametrize("mode", [0, 1])
def test_many_matches_oracle(nonblocking, oracle_mod, mode, team):
    """team 8: every graph with edges is solved by a team of workgroups (the
    graphs are small next to the per-CU share of all edges); team 1: one
    workgroup per graph."""
    grb = nonblocking
    gs, ogs = _graphs(oracle_mod)
    grb.GrM_set_many_team_max(team)
    try:
        mg = grb.GrM_Multigraph_new([g.AT for g in gs])
    finally:
        grb.GrM_set_many_team_max(8)
    off = grb.GrM_Multigraph_offsets(mg, len(gs))
    assert off[-1] == sum(g.n for g in gs)
    for dtype, tol, bound in ((torch.float64, 1e-10, None), (torch.float32, 1e-6, 1e-5)):
        t = grb.builtin("GrB_FP32" if dtype == torch.float32 else "GrB_FP64")
        X = torch.empty(int(off[-1]), dtype=dtype, device="cuda")
        its, res = grb.GrM_pagerank_many(X, t, mg, len(gs), D, tol, 1000, mode)
        x = X.cpu().numpy().astype(np.float64)
        for i, og in enumerate(ogs):
            xi = x[off[i]:off[i + 1]]
            ref = oracle_mod.pagerank(og, D, fixed_iters=int(its[i]), mode=mode)
            if bound is None:
                assert np.abs(xi - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12, i
                free = oracle_mod.pagerank(og, D, tol=tol, mode=mode)
                assert abs(int(its[i]) - free.iters) <= 1, (i, its[i], free.iters)
                assert abs(res[i] - ref.resid) <= 4 * np.abs(xi - ref.x).sum() + 1e-16
            else:
                assert np.abs(xi - ref.x).sum() <= bound, i
        # replays of the captured launch: identical
        X2 = X.clone()
        its2, res2 = grb.GrM_pagerank_many(X, t, mg, len(gs), D, tol, 1000, mode)
        assert np.array_equal(its, its2) and np.array_equal(res, res2)
        assert torch.equal(X, X2)
    grb.GrM_Multigraph_free(mg)
    for g in gs:
        g.free()


def test_many_rmat_workload_sample(nonblocking, oracle_mod):
    """A slice of the many-graph workload (scales 10-16, seeds 3000+i)."""
    from paper_2509_14211_amd import api
    grb = nonblocking
    specs = synthetic.many_graph_specs(24)
    gs = [api.rmat_graph(s, 16, seed) for s, seed in specs]
    mg = grb.GrM_Multigraph_new([g.AT for g in gs])
    off = grb.GrM_Multigraph_offsets(mg, len(gs))
    X = torch.empty(int(off[-1]), dtype=torch.float32, device="cuda")
    its, res = grb.GrM_pagerank_many(X, grb.builtin("GrB_FP32"), mg, len(gs), D, 1e-6, 1000)
    x = X.cpu().numpy().astype(np.float64)
    assert np.all(res <= 1e-6)
    for i, (s, seed) in enumerate(specs):
        og = oracle_mod.rmat_graph(s, 16, seed)
        ref = oracle_mod.pagerank(og, D, fixed_iters=int(its[i]))
        assert np.abs(x[off[i]:off[i + 1]] - ref.x).sum() <= 1e-5, (i, s)
        assert abs(x[off[i]:off[i + 1]].sum() - 1.0) < 1e-4
    grb.GrM_Multigraph_free(mg)
    for g in gs:
        g.free()


def test_many_errors(nonblocking):
    grb = nonblocking
    for bad in (0, 9):
        with pytest.raises(grb.GrBError):
            grb.GrM_set_many_team_max(bad)
    with pytest.raises(grb.GrBError):
        grb.GrM_Multigraph_new([])
    A = grb.GrB_Matrix_new(grb.builtin("GrB_FP32"), 3, 4)
    with pytest.raises(grb.GrBError) as e:
        grb.GrM_Multigraph_new([A])
    assert e.value.info == -6
    grb.GrB_Matrix_free(A)


def test_many_team_wait_give_up_is_reported(nonblocking, oracle_mod):
    """Failure path of the team barrier, forced from the host with a zero
    wait limit: members give up and exit instead of waiting, the launch
    still completes, GrM_pagerank_many reports GrB_PANIC, and the same
    multigraph then solves correctly with the normal limit."""
    grb = nonblocking
    gs, ogs = _graphs(oracle_mod)
    mg = grb.GrM_Multigraph_new([g.AT for g in gs])
    off = grb.GrM_Multigraph_offsets(mg, len(gs))
    t = grb.builtin("GrB_FP64")
    X = torch.empty(int(off[-1]), dtype=torch.float64, device="cuda")
    grb.GrM_set_many_team_wait(0)
    try:
        with pytest.raises(grb.GrBError) as e:
            grb.GrM_pagerank_many(X, t, mg, len(gs), D, 1e-10, 1000, 1)
        assert e.value.info == grb.GrB_PANIC
    finally:
        grb.GrM_set_many_team_wait(10 ** 9)
    its, res = grb.GrM_pagerank_many(X, t, mg, len(gs), D, 1e-10, 1000, 1)
    x = X.cpu().numpy()
    for i, og in enumerate(ogs):
        ref = oracle_mod.pagerank(og, D, fixed_iters=int(its[i]), mode=1)
        assert np.abs(x[off[i]:off[i + 1]] - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12, i
    grb.GrM_Multigraph_free(mg)
    for g in gs:
        g.free()
