"""Generated fusion of elementwise trees (nonblocking mode): random trees of
eWiseAdd / eWiseMult / apply (bound constants and bound device scalars)
over FP32, FP64 and INT32 vectors give bit for bit the values the oracle's
one-operation-at-a-time evaluation gives (each operation rounded in its own
type, oracle/ewise.py), and the results of the per-operation kernels
(blocking mode); they run as one kernel, and reuse the compiled code from
memory and from the code cache directory."""
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
        ks = [k for k, (_, lt) in enumerate(self.leaves) if lt == t]
        k = ks[self.rng.integers(len(ks))]
        return self.leaves[k][0], ("leaf", k)

    def build(self, depth, n, t):
        """Returns (handle, owned, expression) of a random expression of type
        t (binary operations and binds take operands of their own type; a
        unary apply may convert from FP32, FP64 or INT32); the expression is
        the tree in oracle/ewise.py's notation."""
        g, rng = self.grb, self.rng
        if depth == 0 or rng.random() < 0.2:
            h, e = self.leaf(t)
            return h, False, e
        kind = rng.integers(5)
        out = self.vec(t, n)
        self.nops += 1
        if kind <= 1:
            a, oa, ea = self.build(depth - 1, n, t)
            b, ob, eb = self.build(depth - 1, n, t)
            name = BIN_M[rng.integers(len(BIN_M))]
            op = g.builtin(_opname("b", name, t))
            if kind == 0:
                g.GrB_Vector_eWiseMult_BinaryOp(out, None, None, op, a, b)
            else:
                g.GrB_Vector_eWiseAdd_BinaryOp(out, None, None, op, a, b)
            for h, o in ((a, oa), (b, ob)):
                if o:
                    g.GrB_Vector_free(h)
            return out, True, ("ewise", t, name, ea, eb)
        if kind == 2:
            ct = ["FP32", "FP64", "INT32"][rng.integers(3)]
            if ct == "INT32":
                a, ea = self.leaf(ct)
                oa = False
            else:
                a, oa, ea = self.build(depth - 1, n, ct)
            name = UN[rng.integers(len(UN))]
            g.GrB_Vector_apply(out, None, None, g.builtin(_opname("u", name, t)), a)
            e = ("unary", t, name, ea)
        else:
            a, oa, ea = self.build(depth - 1, n, t)
            name = BIN[rng.integers(len(BIN))]
            op = g.builtin(_opname("b", name, t))
            if kind == 3:
                k = float(rng.uniform(0.5, 2.0))
                if rng.random() < 0.5:
                    g.GrB_Vector_apply_BinaryOp1st_FP64(out, None, None, op, k, a)
                    e = ("bind1st", t, name, k, ea)
                else:
                    g.GrB_Vector_apply_BinaryOp2nd_FP64(out, None, None, op, a, k)
                    e = ("bind2nd", t, name, ea, k)
            else:
                j = int(rng.integers(len(self.scalars)))
                g.GrB_Vector_apply_BinaryOp2nd_Scalar(out, None, None, op, a, self.scalars[j])
                e = ("bind2nd_scalar", t, name, ea, j)
        if oa:
            g.GrB_Vector_free(a)
        return out, True, e


def _leaf_values(n, seed):
    """Host values of the leaves (numpy, in the leaf's type) and the type
    names: FP32 and FP64 random values, small integers, two iso vectors,
    and FP64 multiples of 1/256 (their sum is exact in any order)."""
    rng = np.random.default_rng(seed)
    vals = [rng.uniform(0.5, 2.0, n).astype(np.float32), rng.uniform(-2.0, 2.0, n),
            rng.integers(0, 5, n).astype(np.int32), np.full(n, 1.5), np.full(n, 0.25, np.float32),
            rng.integers(-512, 513, n) / 256.0]
    return vals, ["FP32", "FP64", "INT32", "FP64", "FP32", "FP64"]


ISO_LEAVES = (3, 4)  # held as iso-valued vectors


def _leaves(grb, vals, types):
    from paper_2509_14211_amd import api
    out = []
    for k, (v, t) in enumerate(zip(vals, types)):
        if k in ISO_LEAVES:
            h = grb.GrB_Vector_new(grb.builtin("GrB_" + t), len(v))
            grb.GrM_Vector_fill(h, float(v[0]))
        else:
            h = api.vector_from_tensor(torch.from_numpy(v).cuda())
        out.append((h, t))
    return out


def _scalars(grb, leaf):
    """A host-set scalar, a pending reduction of the dyadic leaf (folded as a
    device value) and an affine map of it."""
    s1 = grb.GrB_Scalar_new(grb.builtin("GrB_FP64"))
    grb.GrB_Scalar_setElement_FP64(s1, 0.75)
    s2 = grb.GrB_Scalar_new(grb.builtin("GrB_FP64"))
    grb.GrB_Vector_reduce_Monoid_Scalar(s2, None, grb.builtin("GrB_PLUS_MONOID_FP64"), leaf)
    s3 = grb.GrB_Scalar_new(grb.builtin("GrB_FP64"))
    grb.GrM_Scalar_affine(s3, 1e-6, s2, 0.25)
    return [s1, s2, s3]


def _run(grb, mode, n, seed, t):
    """(result, operations, expression, leaf values, scalar values) of the
    random tree of this seed, recorded in the given mode."""
    from paper_2509_14211_amd import api
    from oracle import ewise
    grb.GrM_set_mode(mode)
    vals, types = _leaf_values(n, seed)
    leaves = _leaves(grb, vals, types)
    scalars = _scalars(grb, leaves[5][0])
    b = Builder(grb, leaves, scalars, seed)
    root, owned, expr = b.build(4, n, t)
    if not owned:
        root2 = grb.GrB_Vector_new(grb.builtin("GrB_" + t), n)
        grb.GrB_Vector_apply(root2, None, None, grb.builtin(_opname("u", "IDENTITY", t)), root)
        root = root2
        expr = ("unary", t, "IDENTITY", expr)
    out = api.tensor_from_vector(root, torch.float32 if t == "FP32" else torch.float64).cpu()
    for h, _ in leaves:
        grb.GrB_Vector_free(h)
    for s in scalars:
        grb.GrB_Scalar_free(s)
    grb.GrB_Vector_free(root)
    grb.GrM_set_mode(grb.GrB_NONBLOCKING)
    s2 = float(np.sum(vals[5]))  # exact: multiples of 1/256 far below 2^53
    svals = [0.75, s2, ewise.fma_double(1e-6, s2, 0.25)]
    return out, b.nops, expr, vals, svals


def _bits_equal(got, ref, t):
    """Bit for bit, NaN where ref has NaN."""
    got, ref = torch.as_tensor(got), torch.as_tensor(ref)
    if not torch.equal(torch.isnan(got), torch.isnan(ref)):
        return False
    m = ~torch.isnan(ref)
    it = torch.int64 if t == "FP64" else torch.int32
    return torch.equal(got[m].view(it), ref[m].view(it))


@pytest.mark.parametrize("seed", list(range(24)))
def test_random_trees_match_oracle_and_per_op_kernels(gpu, seed):
    from oracle import ewise
    n = 50001 + seed
    t = "FP32" if seed % 2 else "FP64"
    ref, nops, expr, vals, svals = _run(gpu, gpu.GrB_BLOCKING, n, seed, t)
    gpu.GrM_reset_stats()
    got, _, expr2, _, _ = _run(gpu, gpu.GrB_NONBLOCKING, n, seed, t)
    st = gpu.GrM_get_stats()
    assert expr2 == expr
    want = ewise.evaluate(expr, vals, svals, n)
    assert want.dtype == (np.float32 if t == "FP32" else np.float64)
    # the generated kernel against the oracle's definition, then against the
    # per-operation kernels
    assert _bits_equal(got, torch.from_numpy(want), t), (seed, expr)
    assert _bits_equal(got, ref, t), seed
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
        a = _run(gpu, gpu.GrB_NONBLOCKING, 4099, 101, "FP64")[0]
        s1 = gpu.GrM_get_stats()
        assert s1["jit_compiles"] >= 1 and s1["jit_disk_hits"] == 0
        assert any(p.suffix == ".co" for p in tmp_path.iterdir())
        gpu.GrM_code_cache_clear()
        gpu.GrM_reset_stats()
        b = _run(gpu, gpu.GrB_NONBLOCKING, 4099, 101, "FP64")[0]
        s2 = gpu.GrM_get_stats()
        assert s2["jit_compiles"] == 0 and s2["jit_disk_hits"] == s1["jit_compiles"]
        assert torch.equal(torch.nan_to_num(a), torch.nan_to_num(b))
        gpu.GrM_reset_stats()
        _run(gpu, gpu.GrB_NONBLOCKING, 4099, 101, "FP64")
        s3 = gpu.GrM_get_stats()
        assert s3["jit_compiles"] == 0 and s3["jit_disk_hits"] == 0 and s3["jit_memory_hits"] >= 1
    finally:
        del os.environ["NBGRB_CODE_CACHE"]
