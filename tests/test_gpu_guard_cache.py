"""Execution errors of the iterative drivers and the two caches of the
runtime.

* A start vector holding a NaN makes the first pass's L1 residual NaN.  A
  NaN compares false with the tolerance, so without a check the loop would
  stop and report a "converged" NaN vector; the drivers report GrB_PANIC
  instead (the condition is forced from the host by the caller's x0, every
  kernel still exits normally).
* The plan cache (the analogue of the paper's signature-keyed code cache,
  Section III-C): a second solve on the same matrix re-plans nothing; a
  different tile geometry or a different matrix does.
* The autotuner's on-disk choice cache (the analogue of the persistent
  compile cache the paper mentions in Section IV): a later process reuses a
  choice without timing, keyed by a signature that includes the value type,
  and the last line written for a signature wins."""
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

PANIC = -101


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("dangling", [0, 1])
def test_nan_start_vector_is_an_execution_error(nonblocking, oracle_mod, dtype, dangling):
    from paper_2509_14211_amd import api
    grb = nonblocking
    print("nan x0", dtype, "dangling", dangling, flush=True)
    g = api.rmat_graph(11)
    x0 = torch.full((g.n,), 1.0 / g.n, dtype=torch.float64)
    x0[7] = float("nan")
    with pytest.raises(grb.GrBError) as e:
        api.pagerank(g, dtype, tol=1e-9, dangling=dangling, x0=x0)
    assert e.value.info == PANIC
    # the library recovers: the next solve is exact
    x, it, res = api.pagerank(g, torch.float64, tol=1e-9, dangling=dangling)
    og = oracle_mod.rmat_graph(11)
    ref = oracle_mod.pagerank(og, 0.85, fixed_iters=it, mode=dangling)
    xx = x.cpu().numpy()
    assert np.abs(xx - ref.x).sum() / np.abs(ref.x).sum() <= 1e-12
    g.free()


def test_inf_start_vector_in_ppr_is_an_execution_error(nonblocking):
    from paper_2509_14211_amd import api
    grb = nonblocking
    g = api.rmat_graph(10)
    x0 = torch.zeros(g.n, dtype=torch.float32, device="cuda")
    x0[3] = float("inf")
    xv = api.vector_from_tensor(x0)
    with pytest.raises(grb.GrBError) as e:
        api.ppr(g, [3, 9], torch.float32, x0=xv)
    assert e.value.info == PANIC
    grb.GrB_Vector_free(xv)
    x, it, res = api.ppr(g, [3, 9], torch.float32)
    assert it > 0 and res <= 1e-6 and np.isfinite(x.cpu().numpy()).all()
    g.free()


def test_plan_cache_hits_on_repeated_solves(nonblocking):
    from paper_2509_14211_amd import api
    grb = nonblocking
    g = api.rmat_graph(12)
    f32 = grb.builtin("GrB_FP32")
    f64 = grb.builtin("GrB_FP64")
    grb.GrM_Matrix_plan_set(g.AT, f32, None)
    grb.GrM_Matrix_plan_set(g.AT, f64, None)
    grb.GrM_reset_stats()
    api.pagerank(g, torch.float32, tol=1e-6)
    s1 = grb.GrM_get_stats()
    assert s1["plan_misses"] >= 1
    grb.GrM_reset_stats()
    api.pagerank(g, torch.float32, tol=1e-6)
    s2 = grb.GrM_get_stats()
    assert s2["plan_misses"] == 0 and s2["plan_hits"] > 0
    # the tile list depends on the pattern and the tile geometry, not on
    # the value type: the FP64 solve with the same geometry reuses it (the
    # kernels are compiled per type ahead of time)
    grb.GrM_reset_stats()
    api.pagerank(g, torch.float64, tol=1e-9)
    s3 = grb.GrM_get_stats()
    assert s3["plan_misses"] == 0 and s3["plan_hits"] > 0
    # a different geometry misses once, then hits
    cfg = dict(kernel=1, lds_entries=512, lds_rows=256, long_row=512, chunk=512, grid=0, hot=4096,
               relabel=0, xcd_split=0)
    grb.GrM_Matrix_plan_set(g.AT, f32, cfg)
    grb.GrM_reset_stats()
    api.pagerank(g, torch.float32, tol=1e-6)
    s4 = grb.GrM_get_stats()
    assert s4["plan_misses"] == 1
    grb.GrM_reset_stats()
    api.pagerank(g, torch.float32, tol=1e-6)
    assert grb.GrM_get_stats()["plan_misses"] == 0
    # a different matrix with the same shape misses
    g2 = api.rmat_graph(12, seed=99)
    grb.GrM_reset_stats()
    api.pagerank(g2, torch.float32, tol=1e-6)
    assert grb.GrM_get_stats()["plan_misses"] >= 1
    grb.GrM_Matrix_plan_set(g.AT, f32, None)
    g.free()
    g2.free()


def test_autotune_cache_roundtrip(nonblocking, tmp_path):
    from paper_2509_14211_amd import api
    grb = nonblocking
    path = str(tmp_path / "tune.txt")
    f32 = grb.builtin("GrB_FP32")
    f64 = grb.builtin("GrB_FP64")
    g = api.rmat_graph(12)
    plan, us = grb.GrM_autotune_pagerank(g.AT, g.outdeg, f32, path)
    assert us > 0.0
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("pr-fused t%d " % 2)
    assert grb.GrM_Matrix_plan_get(g.AT, f32) == plan
    # a fresh matrix with the same signature (as in a later process): the
    # stored choice is installed without timing any candidate
    g2 = api.rmat_graph(12)
    grb.GrM_reset_stats()
    plan2, us2 = grb.GrM_autotune_pagerank(g2.AT, g2.outdeg, f32, path)
    st = grb.GrM_get_stats()
    assert us2 == -1.0 and plan2 == plan
    assert st["fused_launches"] == 0 and st["kernels"] <= 2
    assert grb.GrM_Matrix_plan_get(g2.AT, f32) == plan
    # the value type is part of the signature: FP64 is timed and stored apart
    plan64, us64 = grb.GrM_autotune_pagerank(g2.AT, g2.outdeg, f64, path)
    assert us64 > 0.0
    lines = open(path).read().splitlines()
    assert len(lines) == 2 and lines[1].startswith("pr-fused t%d " % 3)
    # the last line for a signature wins
    key, fields, _ = lines[0].split("|")
    other = dict(plan)
    other["hot"] = 1024 if plan["hot"] != 1024 else 2048
    other["kernel"] = 1
    other.update(lds_entries=512, lds_rows=256, long_row=512, chunk=512)
    vals = [other[f] for f in ("kernel", "lds_entries", "lds_rows", "long_row", "chunk", "grid", "hot",
                               "relabel", "xcd_split")]
    with open(path, "a") as f:
        f.write("%s|%s|1.0\n" % (key, " ".join(str(v) for v in vals)))
    g3 = api.rmat_graph(12)
    plan3, us3 = grb.GrM_autotune_pagerank(g3.AT, g3.outdeg, f32, path)
    assert us3 == -1.0 and plan3 == other
    x, it, res = api.pagerank(g3, torch.float32, tol=1e-6)
    assert res <= 1e-6
    for h in (g, g2, g3):
        grb.GrM_Matrix_plan_set(h.AT, f32, None)
        grb.GrM_Matrix_plan_set(h.AT, f64, None)
        h.free()
    assert os.path.exists(path)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_guard_reads_do_not_change_the_solve(nonblocking, oracle_mod, dtype):
    """The drivers read the loop guard every check_every passes and keep two
    passes queued behind each read; those passes are skipped on the device
    once the residual reached tol or itermax passes ran.  Every cadence
    gives the same pass count, residual and ranks as checking once at the
    end, the ranks are those of the oracle after that many passes, and no
    more than itermax passes run."""
    from paper_2509_14211_amd import api
    grb = nonblocking
    g = api.rmat_graph(11)
    og = oracle_mod.rmat_graph(11)
    tol = 1e-6 if dtype == torch.float32 else 1e-10
    for itermax in (0, 1, 2, 3, 7, 1000):
        ref_x, ref_it, ref_res = api.pagerank(g, dtype, tol=tol, itermax=itermax, check_every=1000)
        assert ref_it <= itermax
        # no pass: the start vector (every entry 1/n)
        want = (oracle_mod.pagerank(og, 0.85, fixed_iters=ref_it, mode=1).x if ref_it > 0
                else np.full(g.n, 1.0 / g.n))
        ref_np = ref_x.cpu().numpy().astype(np.float64)
        bound = 1e-5 if dtype == torch.float32 else 1e-12
        assert np.abs(ref_np - want).sum() <= bound * max(1.0, np.abs(want).sum())
        for check_every in (1, 2, 3, 5, 8):
            print("itermax", itermax, "check_every", check_every, dtype, flush=True)
            x, it, res = api.pagerank(g, dtype, tol=tol, itermax=itermax, check_every=check_every)
            assert it == ref_it and res == ref_res
            assert torch.equal(x, ref_x)
    g.free()
