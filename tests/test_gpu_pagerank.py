"""Fused (nonblocking) and unfused (blocking) PageRank on the GPU against the
FP64 oracle, plus the closed forms, loop control, determinism and the
launch counts that show the fusion.

Tolerances: FP64 paths agree with the oracle to 1e-12 relative L1 at the
same iteration count; FP32 ranks (FP64 residual and dangling sums) to 1e-5
absolute L1."""
import numpy as np
import pytest
import torch

import synthetic

pytestmark = pytest.mark.gpu

D = 0.85


def _rel_l1(a, b):
    return np.abs(a - b).sum() / np.abs(b).sum()


def _pr(g, dtype, **kw):
    from paper_2509_14211_amd import api
    x, it, res = api.pagerank(g, dtype, **kw)
    return x.cpu().numpy().astype(np.float64), it, res


@pytest.mark.parametrize("scale", [10, 12])
@pytest.mark.parametrize("mode", [0, 1])
def test_fp64_fused_matches_oracle(nonblocking, oracle_mod, scale, mode):
    from paper_2509_14211_amd import api
    print("fp64 fused scale", scale, "mode", mode, flush=True)
    g = api.rmat_graph(scale)
    og = oracle_mod.rmat_graph(scale)
    x, it, res = _pr(g, torch.float64, tol=1e-9, dangling=mode)
    ref = oracle_mod.pagerank(og, D, fixed_iters=it, mode=mode)
    assert _rel_l1(x, ref.x) <= 1e-12
    # rho_k = |x_k - x_{k-1}|_1, so by the triangle inequality it can differ
    # from the oracle's by at most the iterates' errors (~ twice the last).
    assert abs(res - ref.resid) <= 4 * np.abs(x - ref.x).sum() + 1e-16
    free = oracle_mod.pagerank(og, D, tol=1e-9, itermax=1000, mode=mode)
    assert abs(it - free.iters) <= 1
    g.free()


@pytest.mark.parametrize("scale", [12, 16])
def test_fp32_fused_matches_fp64_oracle(nonblocking, oracle_mod, scale):
    from paper_2509_14211_amd import api
    print("fp32 fused scale", scale, flush=True)
    g = api.rmat_graph(scale)
    og = oracle_mod.rmat_graph(scale)
    x, it, res = _pr(g, torch.float32, tol=1e-6)
    ref = oracle_mod.pagerank(og, D, fixed_iters=it, mode=1)
    err = np.abs(x - ref.x).sum()
    assert err <= 1e-5
    assert abs(res - ref.resid) <= 4 * err + 1e-7
    g.free()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_blocking_equals_nonblocking(gpu, oracle_mod, dtype):
    """Mode equivalence (Section II): same iterations, same ranks up to
    reassociation; blocking runs one kernel per operation."""
    from paper_2509_14211_amd import api
    g = api.rmat_graph(11)
    gpu.GrM_set_mode(gpu.GrB_BLOCKING)
    gpu.GrM_reset_stats()
    xb, itb, rb = _pr(g, dtype, tol=1e-9 if dtype == torch.float64 else 1e-6)
    sb = gpu.GrM_get_stats()
    gpu.GrM_set_mode(gpu.GrB_NONBLOCKING)
    gpu.GrM_reset_stats()
    xn, itn, rn = _pr(g, dtype, tol=1e-9 if dtype == torch.float64 else 1e-6)
    sn = gpu.GrM_get_stats()
    assert itb == itn
    tol = 1e-13 if dtype == torch.float64 else 1e-6
    assert np.abs(xb - xn).sum() <= tol
    assert sb["fused_launches"] == 0
    assert sn["fused_launches"] >= itn
    # blocking: 7 kernels per pass (mult, mxv, affine, apply, absdiff, reduce,
    # masked reduce); nonblocking: one fused pass per iteration.
    assert sb["kernels"] >= 7 * itb
    assert sn["kernels"] <= sn["fused_launches"] + 12
    g.free()


def test_repeatable_and_check_interval_invariant(nonblocking):
    from paper_2509_14211_amd import api
    g = api.rmat_graph(12)
    a = _pr(g, torch.float32, tol=1e-6, check_every=1)
    b = _pr(g, torch.float32, tol=1e-6, check_every=8)
    c = _pr(g, torch.float32, tol=1e-6, check_every=8)
    assert a[1] == b[1] == c[1]
    assert np.array_equal(a[0], b[0]) and np.array_equal(b[0], c[0])
    assert a[2] == b[2] == c[2]
    g.free()


def test_itermax_and_zero_passes(nonblocking, oracle_mod):
    from paper_2509_14211_amd import api
    g = api.rmat_graph(10)
    og = oracle_mod.rmat_graph(10)
    x, it, res = _pr(g, torch.float64, tol=1e-12, itermax=3)
    assert it == 3 and res > 1e-12
    ref = oracle_mod.pagerank(og, D, fixed_iters=3)
    assert _rel_l1(x, ref.x) <= 1e-12
    x, it, res = _pr(g, torch.float64, tol=1.5, itermax=10)
    assert it == 0 and res == 1.0
    assert np.allclose(x, 1.0 / g.n, rtol=0, atol=0)
    x, it, res = _pr(g, torch.float64, tol=1e-9, itermax=0)
    assert it == 0
    g.free()


def test_warm_start_x0(nonblocking, oracle_mod):
    from paper_2509_14211_amd import api
    g = api.rmat_graph(11)
    og = oracle_mod.rmat_graph(11)
    x0 = synthetic.random_distribution(g.n, 5)
    x, it, res = _pr(g, torch.float64, tol=1e-10, x0=torch.from_numpy(x0))
    ref = oracle_mod.pagerank(og, D, fixed_iters=it, x0=x0)
    assert _rel_l1(x, ref.x) <= 1e-12
    g.free()


# ------------------------------------------------------------ closed forms / edges

def _graph(spec):
    from paper_2509_14211_amd import api
    n, src, dst = spec
    return api.graph_from_edges(n, src, dst)


@pytest.mark.parametrize("m", [3, 700, 20000])
def test_stars_closed_form(nonblocking, m):
    """m = 700 exercises whole-row tiles, m = 20000 split hub rows."""
    n = m + 1
    g = _graph(synthetic.star_in(m))
    x, _, _ = _pr(g, torch.float64, tol=1e-14, itermax=500)
    assert abs(x[0] - (1 + m * D) / (m + 1 + m * D)) < 1e-13
    assert np.allclose(x[1:], 1 / (m + 1 + m * D), rtol=1e-12, atol=0)
    g.free()
    g = _graph(synthetic.star_out(m))
    x, _, _ = _pr(g, torch.float64, tol=1e-14, itermax=500)
    assert abs(x[0] - 1 / (n + D)) < 1e-13
    assert np.allclose(x[1:], (m + D) / (m * (n + D)), rtol=1e-12, atol=0)
    g.free()
    g = _graph(synthetic.star_both(m))
    x, _, _ = _pr(g, torch.float64, tol=1e-14, itermax=500)
    assert abs(x[0] - (1 + D * m) / (n * (1 + D))) < 1e-13
    assert np.allclose(x[1:], (D + m) / (m * n * (1 + D)), rtol=1e-12, atol=0)
    g.free()


def test_star_residual_sequence(nonblocking):
    """From the uniform start the bidirectional star's residual is exactly
    2 (m-1) d^t / n; the iteration count follows from it."""
    m = 50
    n = m + 1
    g = _graph(synthetic.star_both(m))
    for k in (1, 2, 5, 17):
        _, it, res = _pr(g, torch.float64, tol=0.0, itermax=k)
        assert it == k
        assert abs(res - 2 * (m - 1) * D ** k / n) <= 1e-12 * res
    g.free()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_small_graphs(nonblocking, dtype):
    eps = 1e-14 if dtype == torch.float64 else 1e-6
    g = _graph(synthetic.cycle(37))
    x, it, _ = _pr(g, dtype, tol=1e-12 if dtype == torch.float64 else 1e-6)
    assert it == 1 and np.allclose(x, 1 / 37, rtol=eps, atol=0)
    g.free()
    g = _graph(synthetic.empty(9))
    x, _, _ = _pr(g, dtype, tol=1e-12, itermax=50)
    assert np.allclose(x, 1 / 9, rtol=eps, atol=0)
    x, _, _ = _pr(g, dtype, tol=1e-12, itermax=50, dangling=0)
    assert np.allclose(x, (1 - D) / 9, rtol=eps * 10, atol=0)
    g.free()
    g = _graph(synthetic.empty(1))
    x, _, _ = _pr(g, dtype, tol=1e-12, itermax=50)
    assert abs(x[0] - 1.0) <= eps
    g.free()
    g = _graph(synthetic.path2())
    x, _, _ = _pr(g, dtype, tol=1e-13, itermax=500)
    assert np.allclose(x, [1 / (2 + D), (1 + D) / (2 + D)], rtol=10 * eps, atol=0)
    g.free()


# ------------------------------------------------------------ the Fig. 6 call sequence

def fig6_loop(grb, g, T, damping, tol, itermax):
    """The paper's PageRank loop written as GrB calls, with the residual
    read on the host every iteration (Fig. 6; uniform dangling mass)."""
    n = g.n
    sfx = "FP64" if T == "GrB_FP64" else "FP32"
    typ = grb.builtin(T)
    d = grb.GrB_Vector_new(typ, n)
    grb.GrB_Vector_apply(d, None, None, grb.builtin("GrM_MINV_OR_ZERO_" + sfx), g.outdeg)
    grb.GrB_Vector_apply_BinaryOp1st_FP64(d, None, None, grb.builtin("GrB_TIMES_" + sfx), damping, d)
    r = grb.GrB_Vector_new(typ, n)
    grb.GrM_Vector_fill(r, 1.0 / n)
    Dm = grb.GrB_Scalar_new(grb.builtin("GrB_FP64"))
    desc_c = grb.builtin("GrB_DESC_C")
    plus_m = grb.builtin("GrB_PLUS_MONOID_FP64")
    grb.GrM_Vector_reduce_masked_Scalar(Dm, d, plus_m, r, desc_c)
    rdiff, it = 1.0, 0
    while it < itermax and rdiff > tol:
        t = grb.GrB_Vector_dup(r)
        w = grb.GrB_Vector_new(typ, n)
        grb.GrB_Vector_eWiseMult_BinaryOp(w, None, None, grb.builtin("GrB_TIMES_" + sfx), t, d)
        s = grb.GrB_Vector_new(typ, n)
        grb.GrB_mxv(s, None, None, grb.builtin("GrM_PLUS_SECOND_SEMIRING_" + sfx), g.AT, w)
        c = grb.GrB_Scalar_new(grb.builtin("GrB_FP64"))
        grb.GrM_Scalar_affine(c, damping / n, Dm, (1 - damping) / n)
        grb.GrB_Vector_apply_BinaryOp2nd_Scalar(r, None, None, grb.builtin("GrB_PLUS_" + sfx), s, c)
        tt = grb.GrB_Vector_new(typ, n)
        grb.GrB_Vector_eWiseAdd_BinaryOp(tt, None, None, grb.builtin("GrM_ABSDIFF_" + sfx), t, r)
        rs = grb.GrB_Scalar_new(grb.builtin("GrB_FP64"))
        grb.GrB_Vector_reduce_Monoid_Scalar(rs, None, plus_m, tt)
        grb.GrM_Vector_reduce_masked_Scalar(Dm, d, plus_m, r, desc_c)
        for h in (w, s, tt, t):
            grb.GrB_Vector_free(h)
        grb.GrB_Scalar_free(c)
        rdiff = grb.GrB_Scalar_extractElement_FP64(rs)
        grb.GrB_Scalar_free(rs)
        it += 1
    grb.GrB_Vector_free(d)
    grb.GrB_Scalar_free(Dm)
    return r, it, rdiff


@pytest.mark.parametrize("mode", ["nonblocking", "blocking"])
def test_fig6_call_sequence(gpu, oracle_mod, mode):
    from paper_2509_14211_amd import api
    gpu.GrM_set_mode(gpu.GrB_NONBLOCKING if mode == "nonblocking" else gpu.GrB_BLOCKING)
    g = api.rmat_graph(11)
    og = oracle_mod.rmat_graph(11)
    gpu.GrM_reset_stats()
    r, it, rd = fig6_loop(gpu, g, "GrB_FP64", D, 1e-9, 1000)
    st = gpu.GrM_get_stats()
    x = api.tensor_from_vector(r, torch.float64).cpu().numpy()
    gpu.GrB_Vector_free(r)
    ref = oracle_mod.pagerank(og, D, fixed_iters=it)
    assert _rel_l1(x, ref.x) <= 1e-12
    assert abs(rd - ref.resid) <= 4 * np.abs(x - ref.x).sum() + 1e-16
    if mode == "nonblocking":
        # one fused pass per iteration; the pre-scale runs on its own only in
        # the first iteration (later ones gather the pass's side output)
        assert st["fused_launches"] == it
        assert st["kernels"] <= it + 8
        assert st["elided_nodes"] >= 2 * it
    else:
        assert st["fused_launches"] == 0
        assert st["kernels"] >= 7 * it
    gpu.GrM_set_mode(gpu.GrB_NONBLOCKING)
    g.free()


@pytest.mark.parametrize("mode", ["nonblocking", "blocking"])
def test_fig1_fig2_elementwise(gpu, mode):
    """z = x .* y and z = x .* (y + 1) (Figs. 1 and 2)."""
    gpu.GrM_set_mode(gpu.GrB_NONBLOCKING if mode == "nonblocking" else gpu.GrB_BLOCKING)
    from paper_2509_14211_amd import api
    n = 100003
    xs = torch.from_numpy(synthetic.random_vector(n, 1)).cuda()
    ys = torch.from_numpy(synthetic.random_vector(n, 2)).cuda()
    x = api.vector_from_tensor(xs)
    y = api.vector_from_tensor(ys)
    z = gpu.GrB_Vector_new(gpu.builtin("GrB_FP64"), n)
    gpu.GrB_Vector_eWiseMult_BinaryOp(z, None, None, gpu.builtin("GrB_TIMES_FP64"), x, y)
    zz = api.tensor_from_vector(z, torch.float64)
    assert torch.equal(zz, xs * ys)
    y1 = gpu.GrB_Vector_new(gpu.builtin("GrB_FP64"), n)
    gpu.GrB_Vector_apply_BinaryOp2nd_FP64(y1, None, None, gpu.builtin("GrB_PLUS_FP64"), y, 1.0)
    gpu.GrB_Vector_eWiseMult_BinaryOp(z, None, None, gpu.builtin("GrB_TIMES_FP64"), x, y1)
    gpu.GrB_Vector_free(y1)
    zz = api.tensor_from_vector(z, torch.float64)
    assert torch.equal(zz, xs * (ys + 1.0))
    for h in (x, y, z):
        gpu.GrB_Vector_free(h)
    gpu.GrM_set_mode(gpu.GrB_NONBLOCKING)


def test_errors_surface(nonblocking):
    grb = nonblocking
    f32 = grb.builtin("GrB_FP32")
    f64 = grb.builtin("GrB_FP64")
    a = grb.GrB_Vector_new(f32, 10)
    b = grb.GrB_Vector_new(f64, 10)
    c = grb.GrB_Vector_new(f32, 11)
    with pytest.raises(grb.GrBError) as e:
        grb.GrB_Vector_eWiseAdd_BinaryOp(a, None, None, grb.builtin("GrB_PLUS_FP32"), a, b)
    assert e.value.info == -5
    with pytest.raises(grb.GrBError) as e:
        grb.GrB_Vector_eWiseAdd_BinaryOp(a, None, None, grb.builtin("GrB_PLUS_FP32"), a, c)
    assert e.value.info == -6
    with pytest.raises(grb.GrBError) as e:
        grb.GrB_Vector_eWiseAdd_BinaryOp(a, b, None, grb.builtin("GrB_PLUS_FP32"), a, a)
    assert e.value.info == -8
    s = grb.GrB_Scalar_new(f64)
    assert grb.GrB_Scalar_extractElement_FP64(s) is None
    grb.GrB_Scalar_setElement_FP64(s, 2.5)
    assert grb.GrB_Scalar_extractElement_FP64(s) == 2.5
    for h in (a, b, c):
        grb.GrB_Vector_free(h)
    grb.GrB_Scalar_free(s)
