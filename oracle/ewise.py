"""Plain reference for elementwise expression trees on full vectors, with the
rounding of each operation in its own type (test infrastructure only).

The paper's nonblocking mode fuses a tree of elementwise methods into one
generated loop (Section III-B/C) and requires the same values as running
the methods one by one (Section II: a pending method computes what the
blocking method would have).  On full vectors each method is one IEEE
operation per entry in the type of its output, applied to operands
converted to that type; this module writes that out with numpy arrays of
the stated dtype, one operation at a time.  Only the test suite imports it.

An expression is a nested tuple:
  ("leaf", k)                          leaves[k], a numpy array whose dtype
                                       is the leaf's type (an iso-valued
                                       vector is the array of its value)
  ("ewise", T, op, a, b)               op(a, b) in type T (eWiseAdd and
                                       eWiseMult agree on full vectors)
  ("unary", T, op, a)                  op((T) a)
  ("bind1st", T, op, k, a)             op((T) k, a), k a Python float
  ("bind2nd", T, op, a, k)             op(a, (T) k)
  ("bind2nd_scalar", T, op, a, s)      op(a, (T) scalars[s])
T is "FP32" or "FP64"; operands of a binary operation are converted to T
first.  The operators are the library's closed set (include/nbgrb.h):
MAX(x, y) = x > y ? x : y and MIN(x, y) = x < y ? x : y (so a NaN x yields
y), ABSDIFF(x, y) = |x - y|, MINV(x) = 1 / x, MINV_OR_ZERO(x) = x != 0 ?
1 / x : 0.

Pins: tests/test_oracle_ewise.py evaluates random trees element by element
with Python's own double arithmetic (FP64) and with double arithmetic
rounded to binary32 after every operation (FP32: for +, -, *, / the double
result of binary32 operands rounds to the correctly rounded binary32 result,
since 53 >= 2 * 24 + 2), and checks the operator definitions on hand-picked
values, NaN and infinity included.
"""
from __future__ import annotations

import numpy as np

DTYPES = {"FP32": np.float32, "FP64": np.float64}


def binop(op: str, x, y):
    """The library's binary operator on arrays of one dtype."""
    with np.errstate(all="ignore"):
        if op == "PLUS":
            return x + y
        if op == "MINUS":
            return x - y
        if op == "TIMES":
            return x * y
        if op == "DIV":
            return x / y
        if op == "MAX":
            return np.where(x > y, x, y)
        if op == "MIN":
            return np.where(x < y, x, y)
        if op == "FIRST":
            return x
        if op == "SECOND":
            return y
        if op == "ABSDIFF":
            return np.abs(x - y)
    raise ValueError(op)


def unop(op: str, x):
    """The library's unary operator on an array."""
    one = x.dtype.type(1)
    zero = x.dtype.type(0)
    with np.errstate(all="ignore"):
        if op == "IDENTITY":
            return x
        if op == "ABS":
            return np.abs(x)
        if op == "AINV":
            return -x
        if op == "MINV":
            return one / x
        if op == "MINV_OR_ZERO":
            return np.where(x != zero, one / np.where(x != zero, x, one), zero)
    raise ValueError(op)


def convert(x, T: str):
    """x (an array of any of the leaf types) as an array of type T, rounded
    to nearest."""
    return np.asarray(x).astype(DTYPES[T])


def evaluate(expr, leaves, scalars, n: int):
    """Value of the expression tree as a numpy array of its root's type."""
    kind = expr[0]
    if kind == "leaf":
        return np.asarray(leaves[expr[1]])
    T = expr[1]
    dt = DTYPES[T]
    if kind == "ewise":
        a = convert(evaluate(expr[3], leaves, scalars, n), T)
        b = convert(evaluate(expr[4], leaves, scalars, n), T)
        return binop(expr[2], a, b).astype(dt)
    if kind == "unary":
        a = convert(evaluate(expr[3], leaves, scalars, n), T)
        return unop(expr[2], a).astype(dt)
    if kind == "bind1st":
        a = convert(evaluate(expr[4], leaves, scalars, n), T)
        return binop(expr[2], np.full(n, dt(expr[3]), dtype=dt), a).astype(dt)
    if kind == "bind2nd":
        a = convert(evaluate(expr[3], leaves, scalars, n), T)
        return binop(expr[2], a, np.full(n, dt(expr[4]), dtype=dt)).astype(dt)
    if kind == "bind2nd_scalar":
        a = convert(evaluate(expr[3], leaves, scalars, n), T)
        return binop(expr[2], a, np.full(n, dt(scalars[expr[4]]), dtype=dt)).astype(dt)
    raise ValueError(kind)


def fma_double(a: float, b: float, c: float) -> float:
    """a * b + c with one rounding to double (exact rational arithmetic,
    then Python's correctly rounded conversion)."""
    from fractions import Fraction
    return float(Fraction(a) * Fraction(b) + Fraction(c))
