"""Pins of oracle/ewise.py (elementwise trees with per-operation rounding):
the operator definitions on hand-picked values, NaN and infinity included;
random trees against an element-by-element evaluation in Python's own
double arithmetic (FP64), and in double arithmetic rounded to binary32
after every operation (FP32: the double result of +, -, *, / on binary32
operands rounds to the correctly rounded binary32 result, because
53 >= 2 * 24 + 2); and the single-rounding fused multiply-add."""
import math

import numpy as np
import pytest

from oracle import ewise

BIN = ["PLUS", "MINUS", "TIMES", "DIV", "MAX", "MIN", "FIRST", "SECOND", "ABSDIFF"]
UN = ["IDENTITY", "ABS", "AINV", "MINV", "MINV_OR_ZERO"]
INF, NAN = math.inf, math.nan


def _same(a, b):
    return (math.isnan(a) and math.isnan(b)) or (a == b and math.copysign(1, a) == math.copysign(1, b))


@pytest.mark.parametrize("T", ["FP32", "FP64"])
def test_operator_table(T):
    dt = ewise.DTYPES[T]
    cases = {  # no key differs from another only in the sign of a zero
        ("PLUS", 1.5, 2.25): 3.75, ("MINUS", 1.0, 4.0): -3.0, ("TIMES", -2.0, 0.5): -1.0,
        ("DIV", 1.0, 0.0): INF, ("DIV", -1.0, 0.0): -INF, ("DIV", 0.0, 0.0): NAN, ("DIV", 3.0, -2.0): -1.5,
        ("MAX", 1.0, 2.0): 2.0, ("MAX", NAN, 2.0): 2.0, ("MAX", 2.0, NAN): NAN, ("MAX", -0.0, 0.0): 0.0,
        ("MIN", 1.0, 2.0): 1.0, ("MIN", NAN, 2.0): 2.0, ("MIN", 2.0, NAN): NAN,
        ("FIRST", 7.0, NAN): 7.0, ("SECOND", NAN, 7.0): 7.0,
        ("ABSDIFF", 1.0, 3.5): 2.5, ("ABSDIFF", INF, INF): NAN, ("PLUS", INF, -INF): NAN,
    }
    for (op, x, y), want in cases.items():
        got = float(ewise.binop(op, np.array([x], dt), np.array([y], dt))[0])
        assert _same(got, want), (T, op, x, y, got)
    # a list, not a dict: 0.0 and -0.0 are equal keys
    ucases = [(("ABS", -2.0), 2.0), (("AINV", 3.0), -3.0), (("AINV", 0.0), -0.0), (("MINV", 4.0), 0.25),
              (("MINV", 0.0), INF), (("MINV", -0.0), -INF), (("MINV_OR_ZERO", 0.0), 0.0),
              (("MINV_OR_ZERO", -0.0), 0.0), (("MINV_OR_ZERO", 8.0), 0.125), (("IDENTITY", NAN), NAN)]
    for (op, x), want in ucases:
        got = float(ewise.unop(op, np.array([x], dt))[0])
        assert _same(got, want), (T, op, x, got)


def _r32(x):
    return float(np.float32(x))


def _pdiv(x, y):
    if y == 0.0:
        if x == 0.0 or math.isnan(x):
            return NAN
        return math.copysign(INF, x) * math.copysign(1.0, y)
    return x / y


def _pbin(op, x, y):
    if op == "PLUS":
        return x + y
    if op == "MINUS":
        return x - y
    if op == "TIMES":
        return x * y
    if op == "DIV":
        return _pdiv(x, y)
    if op == "MAX":
        return x if x > y else y
    if op == "MIN":
        return x if x < y else y
    if op == "FIRST":
        return x
    if op == "SECOND":
        return y
    return abs(x - y)


def _pun(op, x):
    if op == "IDENTITY":
        return x
    if op == "ABS":
        return abs(x)
    if op == "AINV":
        return -x
    if op == "MINV":
        return _pdiv(1.0, x)
    return _pdiv(1.0, x) if x != 0.0 else 0.0


def _elem(expr, leaves, scalars, i):
    """One entry of the tree with Python floats, rounding to binary32 after
    every FP32 operation and conversion."""
    kind = expr[0]
    if kind == "leaf":
        return float(leaves[expr[1]][i])
    T = expr[1]
    rnd = _r32 if T == "FP32" else (lambda z: z)
    if kind == "ewise":
        a = rnd(_elem(expr[3], leaves, scalars, i))
        b = rnd(_elem(expr[4], leaves, scalars, i))
        return rnd(_pbin(expr[2], a, b))
    if kind == "unary":
        return rnd(_pun(expr[2], rnd(_elem(expr[3], leaves, scalars, i))))
    if kind == "bind1st":
        return rnd(_pbin(expr[2], rnd(expr[3]), rnd(_elem(expr[4], leaves, scalars, i))))
    if kind == "bind2nd":
        return rnd(_pbin(expr[2], rnd(_elem(expr[3], leaves, scalars, i)), rnd(expr[4])))
    return rnd(_pbin(expr[2], rnd(_elem(expr[3], leaves, scalars, i)), rnd(scalars[expr[4]])))


def _random_tree(rng, T, depth, ltypes):
    if depth == 0 or rng.random() < 0.2:
        ks = [k for k, t in enumerate(ltypes) if t == T]
        return ("leaf", ks[rng.integers(len(ks))])
    kind = rng.integers(5)
    if kind <= 1:
        return ("ewise", T, BIN[rng.integers(len(BIN))], _random_tree(rng, T, depth - 1, ltypes),
                _random_tree(rng, T, depth - 1, ltypes))
    if kind == 2:
        ct = ["FP32", "FP64", "INT32"][rng.integers(3)]
        sub = ("leaf", ltypes.index("INT32")) if ct == "INT32" else _random_tree(rng, ct, depth - 1, ltypes)
        return ("unary", T, UN[rng.integers(len(UN))], sub)
    op = BIN[rng.integers(len(BIN) - 1)]
    sub = _random_tree(rng, T, depth - 1, ltypes)
    if kind == 3:
        k = float(rng.uniform(0.5, 2.0))
        return ("bind1st", T, op, k, sub) if rng.random() < 0.5 else ("bind2nd", T, op, sub, k)
    return ("bind2nd_scalar", T, op, sub, int(rng.integers(3)))


@pytest.mark.parametrize("seed", range(40))
def test_random_trees_match_elementwise_python(seed):
    rng = np.random.default_rng(seed)
    n = 257
    leaves = [rng.uniform(0.5, 2.0, n).astype(np.float32), rng.uniform(-2.0, 2.0, n),
              rng.integers(0, 5, n).astype(np.int32), np.full(n, 1.5), np.full(n, 0.25, np.float32)]
    ltypes = ["FP32", "FP64", "INT32", "FP64", "FP32"]
    scalars = [0.75, float(rng.uniform(-3, 3)), 0.1]
    T = "FP32" if seed % 2 else "FP64"
    expr = _random_tree(rng, T, 4, ltypes)
    got = ewise.evaluate(expr, leaves, scalars, n)
    assert got.dtype == ewise.DTYPES[T]
    for i in range(n):
        want = _elem(expr, leaves, scalars, i)
        assert _same(float(got[i]), want), (seed, i, float(got[i]), want, expr)


def test_fma_is_one_rounding():
    a = 1.0 + 2.0 ** -30
    c = -(1.0 + 2.0 ** -29)
    assert a * a + c == 0.0                     # two roundings lose the low term
    assert ewise.fma_double(a, a, c) == 2.0 ** -60
    assert ewise.fma_double(1e-6, 3.0, 0.25) == 0.250003
