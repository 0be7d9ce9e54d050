"""Generated fusion of elementwise trees (nonblocking mode): random trees of
eWiseAdd / eWiseMult / apply (bound constants and bound device scalars)
over FP32, FP64 and INT32 vectors give bit-for-bit the results of the
per-operation kernels (blocking mode), run as one kernel, and reuse the
compiled code from memory and from the code cache directory."""
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

BIN = ["PLUS", "MINUS", "TIMES", "DIV", "MAX", "MIN", "FIRST", "SECOND"]
BIN_M = BIN + ["ABSDIFF"]
UN = ["IDENTITY", "ABS", "AINV", "MINV", "MINV_OR_ZERO"]


def _opname(kind, name, t):
    pre = "GrM_" if name in ("ABSDIFF", "MINV_OR_ZERO") else "GrB_"
    return pre + name + ("_FP32" if t == "FP32" else "_FP64")


class Builder:
    """Records the same random tree of operations in either mode; every
    intermediate handle is freed as soon as its consumer is recorded, so in
    nonblocking mode only the root is referenced."""

    def __init__(self, grb, leaves, scalars, seed):
        self.grb = grb
        self.leaves = leaves      # list of (handle, type name)
        self.scalars = scalars    # list of GrB_Scalar handles
        self.rng = np.random.default_rng(seed)
        self.nops = 0

    def vec(self, t, n):
        return self.grb.GrB_Vector_new(self.grb.builtin("GrB_" + t), n)

    def leaf(self, t):
        hs = [h for h, lt in self.leaves if lt == t]
        return hs[self.rng.integers(len(hs))]

    def build(self, depth, n, t):
        """Returns (handle, owned) of a random expression of type t (binary
        operations and binds take operands of their own type; a unary apply
        may convert from FP32, FP64 or INT32)."""
        g, rng = self.grb, self.rng
        if depth == 0 or rng.random() < 0.2:
            return self.leaf(t), False
        kind = rng.integers(5)
        out = self.vec(t, n)
        self.nops += 1
        if kind <= 1:
            a, oa = self.build(depth - 1, n, t)
            b, ob = self.build(depth - 1, n, t)
            op = g.builtin(_opname("b", BIN_M[rng.integers(len(BIN_M))], t))
            if kind == 0:
                g.GrB_Vector_eWiseMult_BinaryOp(out, None, None, op, a, b)
            else:
                g.GrB_Vector_eWiseAdd_BinaryOp(out, None, None, op, a, b)
            for h, o in ((a, oa), (b, ob)):
                if o:
                    g.GrB_Vector_free(h)
            return out, True
        if kind == 2:
            ct = ["FP32", "FP64", "INT32"][rng.integers(3)]
            a, oa = (self.leaf(ct), False) if ct == "INT32" else self.build(depth - 1, n, ct)
            g.GrB_Vector_apply(out, None, None, g.builtin(_opname("u", UN[rng.integers(len(UN))], t)), a)
        else:
            a, oa = self.build(depth - 1, n, t)
            op = g.builtin(_opname("b", BIN[rng.integers(len(BIN))], t))
            if kind == 3:
                k = float(rng.uniform(0.5, 2.0))
                if rng.random() < 0.5:
                    g.GrB_Vector_apply_BinaryOp1st_FP64(out, None, None, op, k, a)
                else:
                    g.GrB_Vector_apply_BinaryOp2nd_FP64(out, None, None, op, a, k)
            else:
                s = self.scalars[rng.integers(len(self.scalars))]
                g.GrB_Vector_apply_BinaryOp2nd_Scalar(out, None, None, op, a, s)
        if oa:
            g.GrB_Vector_free(a)
        return out, True


def _leaves(grb, n, seed):
    from paper_2509_14211_amd import api
    rng = np.random.default_rng(seed)
    x32 = torch.tensor(rng.uniform(0.5, 2.0, n), dtype=torch.float32, device="cuda")
    x64 = torch.tensor(rng.uniform(-2.0, 2.0, n), dtype=torch.float64, device="cuda")
    xi = torch.tensor(rng.integers(0, 5, n), dtype=torch.int32, device="cuda")
    iso64 = grb.GrB_Vector_new(grb.builtin("GrB_FP64"), n)
    grb.GrM_Vector_fill(iso64, 1.5)
    iso32 = grb.GrB_Vector_new(grb.builtin("GrB_FP32"), n)
    grb.GrM_Vector_fill(iso32, 0.25)
    return [(api.vector_from_tensor(x32), "FP32"), (api.vector_from_tensor(x64), "FP64"),
            (api.vector_from_tensor(xi), "INT32"), (iso64, "FP64"), (iso32, "FP32")]


def _scalars(grb, leaf):
    """A host-set scalar and a pending reduction (folded as a device value)."""
    s1 = grb.GrB_Scalar_new(grb.builtin("GrB_FP64"))
    grb.GrB_Scalar_setElement_FP64(s1, 0.75)
    s2 = grb.GrB_Scalar_new(grb.builtin("GrB_FP64"))
    grb.GrB_Vector_reduce_Monoid_Scalar(s2, None, grb.builtin("GrB_PLUS_MONOID_FP64"), leaf)
    s3 = grb.GrB_Scalar_new(grb.builtin("GrB_FP64"))
    grb.GrM_Scalar_affine(s3, 1e-6, s2, 0.25)
    return [s1, s2, s3]


def _run(grb, mode, n, seed, t):
    from paper_2509_14211_amd import api
    grb.GrM_set_mode(mode)
    leaves = _leaves(grb, n, seed)
    scalars = _scalars(grb, leaves[1][0])
    b = Builder(grb, leaves, scalars, seed)
    root, owned = b.build(4, n, t)
    if not owned:
        root2 = grb.GrB_Vector_new(grb.builtin("GrB_" + t), n)
        grb.GrB_Vector_apply(root2, None, None, grb.builtin(_opname("u", "IDENTITY", t)), root)
        root = root2
    out = api.tensor_from_vector(root, torch.float32 if t == "FP32" else torch.float64).cpu()
    for h, _ in leaves:
        grb.GrB_Vector_free(h)
    for s in scalars:
        grb.GrB_Scalar_free(s)
    grb.GrB_Vector_free(root)
    grb.GrM_set_mode(grb.GrB_NONBLOCKING)
    return out, b.nops


@pytest.mark.parametrize("seed", list(range(12)))
def test_random_trees_equal_per_op_kernels(gpu, seed):
    n = 50001 + seed
    t = "FP32" if seed % 2 else "FP64"
    ref, nops = _run(gpu, gpu.GrB_BLOCKING, n, seed, t)
    gpu.GrM_reset_stats()
    got, _ = _run(gpu, gpu.GrB_NONBLOCKING, n, seed, t)
    st = gpu.GrM_get_stats()
    # bit for bit, NaN where the per-op kernels give NaN
    assert torch.equal(torch.isnan(got), torch.isnan(ref))
    m = ~torch.isnan(ref)
    assert torch.equal(got[m].view(torch.int64 if t == "FP64" else torch.int32),
                       ref[m].view(torch.int64 if t == "FP64" else torch.int32)), seed
    if nops >= 2:
        assert st["ewise_fused"] >= 1 and st["ewise_ops"] >= 2


def test_chain_is_one_kernel_and_matches_definition(gpu, oracle_mod):
    """w = |x .* (y + 1) - 2 z| / 3 with intermediates freed: one generated
    launch (fusion 1) against five per-op launches (fusion 0), the same bits,
    and the FP64 definition within rounding."""
    from paper_2509_14211_amd import api
    n = 1 << 20
    rng = np.random.default_rng(5)
    xs, ys, zs = (rng.uniform(-1, 1, n) for _ in range(3))

    def chain():
        g = gpu
        f = g.builtin
        x, y, z = (api.vector_from_tensor(torch.tensor(a, device="cuda")) for a in (xs, ys, zs))
        t1 = g.GrB_Vector_new(f("GrB_FP64"), n)
        g.GrB_Vector_apply_BinaryOp2nd_FP64(t1, None, None, f("GrB_PLUS_FP64"), y, 1.0)
        t2 = g.GrB_Vector_new(f("GrB_FP64"), n)
        g.GrB_Vector_eWiseMult_BinaryOp(t2, None, None, f("GrB_TIMES_FP64"), x, t1)
        t3 = g.GrB_Vector_new(f("GrB_FP64"), n)
        g.GrB_Vector_apply_BinaryOp1st_FP64(t3, None, None, f("GrB_TIMES_FP64"), 2.0, z)
        t4 = g.GrB_Vector_new(f("GrB_FP64"), n)
        g.GrB_Vector_eWiseAdd_BinaryOp(t4, None, None, f("GrM_ABSDIFF_FP64"), t2, t3)
        w = g.GrB_Vector_new(f("GrB_FP64"), n)
        g.GrB_Vector_apply_BinaryOp2nd_FP64(w, None, None, f("GrB_DIV_FP64"), t4, 3.0)
        for h in (t1, t2, t3, t4):
            g.GrB_Vector_free(h)
        out = api.tensor_from_vector(w, torch.float64).cpu().numpy()
        for h in (x, y, z, w):
            g.GrB_Vector_free(h)
        return out

    res = {}
    for level in (0, 1):
        gpu.GrM_set_fusion(level)
        gpu.GrM_reset_stats()
        res[level] = chain()
        res[("k", level)] = gpu.GrM_get_stats()
    gpu.GrM_set_fusion(1)
    assert np.array_equal(res[0], res[1])
    assert res[("k", 1)]["ewise_fused"] == 1 and res[("k", 1)]["ewise_ops"] == 5
    assert res[("k", 0)]["ewise_fused"] == 0
    assert res[("k", 0)]["kernels"] - res[("k", 1)]["kernels"] == 4
    want = np.abs(xs * (ys + 1.0) - 2.0 * zs) / 3.0
    assert np.abs(res[1] - want).max() <= 1e-15 * np.abs(want).max() * 8


def test_reduction_of_a_tree(gpu):
    """sum(|x - (2 y + 1)|): the tree runs as one kernel, then the reduce."""
    from paper_2509_14211_amd import api
    n = 300007
    rng = np.random.default_rng(9)
    xs, ys = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    vals = {}
    for mode in (gpu.GrB_BLOCKING, gpu.GrB_NONBLOCKING):
        gpu.GrM_set_mode(mode)
        f = gpu.builtin
        x, y = (api.vector_from_tensor(torch.tensor(a, device="cuda")) for a in (xs, ys))
        t1 = gpu.GrB_Vector_new(f("GrB_FP64"), n)
        gpu.GrB_Vector_apply_BinaryOp1st_FP64(t1, None, None, f("GrB_TIMES_FP64"), 2.0, y)
        t2 = gpu.GrB_Vector_new(f("GrB_FP64"), n)
        gpu.GrB_Vector_apply_BinaryOp2nd_FP64(t2, None, None, f("GrB_PLUS_FP64"), t1, 1.0)
        t3 = gpu.GrB_Vector_new(f("GrB_FP64"), n)
        gpu.GrB_Vector_eWiseAdd_BinaryOp(t3, None, None, f("GrM_ABSDIFF_FP64"), x, t2)
        for h in (t1, t2):
            gpu.GrB_Vector_free(h)
        s = gpu.GrB_Scalar_new(f("GrB_FP64"))
        gpu.GrB_Vector_reduce_Monoid_Scalar(s, None, f("GrB_PLUS_MONOID_FP64"), t3)
        gpu.GrB_Vector_free(t3)
        gpu.GrM_reset_stats()
        vals[mode] = gpu.GrB_Scalar_extractElement_FP64(s)
        vals[("st", mode)] = gpu.GrM_get_stats()
        for h in (x, y):
            gpu.GrB_Vector_free(h)
        gpu.GrB_Scalar_free(s)
    gpu.GrM_set_mode(gpu.GrB_NONBLOCKING)
    assert vals[gpu.GrB_BLOCKING] == vals[gpu.GrB_NONBLOCKING]
    assert vals[("st", gpu.GrB_NONBLOCKING)]["ewise_fused"] == 1
    assert vals[gpu.GrB_BLOCKING] == pytest.approx(np.abs(xs - (2 * ys + 1)).sum(), rel=1e-12)


def test_code_cache_directory(gpu, tmp_path):
    """A compiled tree is written to the cache directory and loaded from it
    once the in-memory modules are dropped; results do not change."""
    os.environ["NBGRB_CODE_CACHE"] = str(tmp_path)
    try:
        gpu.GrM_code_cache_clear()
        gpu.GrM_reset_stats()
        a, _ = _run(gpu, gpu.GrB_NONBLOCKING, 4099, 101, "FP64")
        s1 = gpu.GrM_get_stats()
        assert s1["jit_compiles"] >= 1 and s1["jit_disk_hits"] == 0
        assert any(p.suffix == ".co" for p in tmp_path.iterdir())
        gpu.GrM_code_cache_clear()
        gpu.GrM_reset_stats()
        b, _ = _run(gpu, gpu.GrB_NONBLOCKING, 4099, 101, "FP64")
        s2 = gpu.GrM_get_stats()
        assert s2["jit_compiles"] == 0 and s2["jit_disk_hits"] == s1["jit_compiles"]
        assert torch.equal(torch.nan_to_num(a), torch.nan_to_num(b))
        gpu.GrM_reset_stats()
        _run(gpu, gpu.GrB_NONBLOCKING, 4099, 101, "FP64")
        s3 = gpu.GrM_get_stats()
        assert s3["jit_compiles"] == 0 and s3["jit_disk_hits"] == 0 and s3["jit_memory_hits"] >= 1
    finally:
        del os.environ["NBGRB_CODE_CACHE"]
