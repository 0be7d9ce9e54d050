"""Plain reference for vectors with missing entries (test infrastructure only).

The paper's vectors are sparse, bitset or full (Section III-A); which
entries are present is part of the value.  This module states the meaning
of the operations on such vectors the slow, obvious way, independent of the
storage format, so that the GPU library can be compared with it whatever
format its estimators choose (Section III-D: estimators never change
results).  Only the test suite imports it.

A vector is ``SVec(n, idx, vals)``: ``idx`` the present positions in
ascending order (int64), ``vals`` their values (float64).  Operators are
named as in the library's binding.

Pins: ``tests/test_oracle_sparse.py`` checks these functions against
brute-force Python sets and dicts on tiny inputs, against scipy's sparse
matrix-vector product, and the breadth-first search built from them against
scipy's shortest-path routine.
"""
from __future__ import annotations

import numpy as np

BINARY = {
    "plus": lambda x, y: x + y,
    "minus": lambda x, y: x - y,
    "times": lambda x, y: x * y,
    "div": lambda x, y: x / y,
    "max": np.maximum,
    "min": np.minimum,
    "first": lambda x, y: x,
    "second": lambda x, y: y,
    "absdiff": lambda x, y: np.abs(x - y),
}

UNARY = {
    "identity": lambda x: x,
    "abs": np.abs,
    "ainv": lambda x: -x,
}


class SVec:
    def __init__(self, n, idx, vals):
        self.n = int(n)
        self.idx = np.asarray(idx, dtype=np.int64)
        self.vals = np.asarray(vals, dtype=np.float64)
        assert self.idx.shape == self.vals.shape
        assert np.all(np.diff(self.idx) > 0)

    @staticmethod
    def full(x):
        x = np.asarray(x, dtype=np.float64)
        return SVec(len(x), np.arange(len(x)), x)

    @staticmethod
    def empty(n):
        return SVec(n, [], [])

    @property
    def nvals(self):
        return len(self.idx)

    def present(self):
        p = np.zeros(self.n, dtype=bool)
        p[self.idx] = True
        return p

    def dense(self, fill=0.0):
        d = np.full(self.n, fill, dtype=np.float64)
        d[self.idx] = self.vals
        return d


def ewise_mult(u: SVec, v: SVec, op: str) -> SVec:
    """Entries present in both u and v: op(u(i), v(i))."""
    both = np.intersect1d(u.idx, v.idx)
    return SVec(u.n, both, BINARY[op](u.dense()[both], v.dense()[both]))


def ewise_add(u: SVec, v: SVec, op: str) -> SVec:
    """Entries present in either: op(u(i), v(i)) where both are, else the
    one that is."""
    pu, pv = u.present(), v.present()
    du, dv = u.dense(), v.dense()
    idx = np.nonzero(pu | pv)[0]
    out = np.where(pu[idx] & pv[idx], BINARY[op](du[idx], dv[idx]), np.where(pu[idx], du[idx], dv[idx]))
    return SVec(u.n, idx, out)


def apply_unary(u: SVec, op: str) -> SVec:
    return SVec(u.n, u.idx, UNARY[op](u.vals))


def apply_bind(u: SVec, op: str, k: float, first: bool) -> SVec:
    """op(k, u(i)) when first, else op(u(i), k), on u's entries."""
    vals = BINARY[op](np.full_like(u.vals, k), u.vals) if first else BINARY[op](u.vals, np.full_like(u.vals, k))
    return SVec(u.n, u.idx, vals)


def reduce(u: SVec) -> float:
    """Sum of the present values (0 when there are none)."""
    return float(np.sum(u.vals))


def _allowed(mask: SVec | None, comp: bool, structural: bool, n: int) -> np.ndarray:
    if mask is None:
        a = np.ones(n, dtype=bool)
    else:
        a = mask.present()
        if not structural:
            a &= mask.dense() != 0
    return ~a if (comp and mask is not None) else a


def _write(w_old: SVec | None, t: SVec, allowed: np.ndarray, replace: bool) -> SVec:
    """w = t on allowed positions; elsewhere w_old's entries unless replace."""
    keep_t = allowed[t.idx]
    idx = [t.idx[keep_t]]
    vals = [t.vals[keep_t]]
    if w_old is not None and not replace:
        keep_o = ~allowed[w_old.idx]
        idx.append(w_old.idx[keep_o])
        vals.append(w_old.vals[keep_o])
    idx = np.concatenate(idx)
    vals = np.concatenate(vals)
    o = np.argsort(idx, kind="stable")
    return SVec(t.n, idx[o], vals[o])


def mxv(rowptr, col, u: SVec, mask: SVec | None = None, comp=False, structural=False, replace=True,
        w_old: SVec | None = None) -> SVec:
    """w(i) = sum of u(j) over the columns j of row i where u(j) is present
    (plus-second on a pattern matrix); w(i) is present when at least one
    such j exists.  A full u gives a full w (an empty row holds 0).  Then
    the mask: w keeps the product on allowed positions and, elsewhere,
    w_old's entries unless replace."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    nrows = len(rowptr) - 1
    pu, du = u.present(), u.dense()
    full = u.nvals == u.n
    idx, vals = [], []
    for i in range(nrows):
        js = col[rowptr[i]:rowptr[i + 1]]
        hit = js[pu[js]]
        if len(hit) or full:
            idx.append(i)
            vals.append(float(np.sum(du[hit])))
    t = SVec(nrows, idx, vals)
    return _write(w_old, t, _allowed(mask, comp, structural, nrows), replace)


def assign_scalar(w_old: SVec | None, n: int, x: float, mask: SVec | None = None, comp=False,
                  structural=False, replace=False) -> SVec:
    """w(i) = x on every allowed position; elsewhere w_old's entries unless
    replace (GrB_Vector_assign with GrB_ALL)."""
    t = SVec(n, np.arange(n), np.full(n, float(x)))
    return _write(w_old, t, _allowed(mask, comp, structural, n), replace)


def bfs_levels(rowptrT, colT, source: int) -> SVec:
    """Breadth-first levels from `source` written with the operations above
    over A^T (rows = destinations): the frontier's successors are
    A^T (+.second) frontier restricted to vertices without a level.  Level
    of the source is 0; unreachable vertices have no entry."""
    n = len(rowptrT) - 1
    levels = SVec.empty(n)
    frontier = SVec(n, [source], [1.0])
    depth = 0
    while frontier.nvals:
        levels = assign_scalar(levels, n, depth, mask=frontier, structural=True)
        frontier = mxv(rowptrT, colT, frontier, mask=levels, comp=True, structural=True, replace=True)
        depth += 1
    return levels
