"""CPU oracle of the learned warm start for personalised PageRank (test
infrastructure only: imported by the tests and the benchmark, never by the
product package).

Everything is plain numpy in FP64.  The pieces, in the order a prediction
runs them:

* ``walk_counts`` -- Monte-Carlo random walks with restart from the seed
  set, drawn from a counter-based SplitMix64 stream so that any other
  implementation of the same definition lands on the same integer counts.
  Walker w starts at seeds[w mod |S|]; at step t it draws u from draw
  key(w, t, 0) and restarts (to seeds[r mod |S|], r = draw key(w, t, 1)) when
  u < 1 - damping or its vertex has no out-edge, otherwise it follows
  out-edge r mod outdeg (r = draw key(w, t, 2)).  key(w, t, j) =
  4 (w T + t - 1) + j, draws are SplitMix64(seed, key), u uses the top 53
  bits.  The walkers' distribution after t steps is the t-th iterate of the
  personalised PageRank map (uniform dangling redistribution) started from
  the teleport vector, which is what makes these counts useful features.
* ``features`` -- 11 per vertex: seed indicator, log(1 + indeg),
  log(1 + outdeg), and log(1 + n c_t / W) for t = 1..8.
* ``forward`` -- two mean-aggregation graph layers over in-neighbours:
  h = ReLU(W1s x_v + W1n mean_in(x) + b1) (11 -> 64), then
  z = w2s . h_v + w2n . mean_in(h) + b2, computed as
  z_v = a_v + mean_in(q) with a = w2s . h + b2 and q = w2n . h (the
  projection commutes with the mean).  An isolated vertex's mean is 0.
* ``softmax`` / ``kl_loss`` -- x0 = softmax(z) over the vertices and
  KL(x* || x0), whose gradient in z is x0 - x*.
* ``backward`` -- gradients of KL(x* || softmax(z)) in every parameter
  (reverse mode of ``forward``, written out by hand).
* ``adam_step`` -- Adam (Kingma & Ba, 2015) with bias correction.

Pins (tests/test_oracle_gnn.py): the SplitMix64 stream against the C
oracle's (itself pinned to a published test vector); walk counts on graphs
where the walk is deterministic (damping 1 on a directed cycle, damping 0)
and, statistically, against the personalised PageRank iterates of the C
oracle; mean aggregation against a dense-matrix product; permutation
equivariance of the forward pass; the softmax/KL gradient identity; every
parameter gradient against central finite differences of ``forward`` +
``kl_loss``; Adam against its closed form on a one-parameter problem.
"""
from __future__ import annotations

import numpy as np

NF = 11          # features per vertex
HID = 64         # hidden width
STEPS = 8        # random-walk feature steps
GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M64 = (1 << 64) - 1

PARAM_SHAPES = (("W1s", (HID, NF)), ("W1n", (HID, NF)), ("b1", (HID,)),
                ("w2s", (HID,)), ("w2n", (HID,)), ("b2", (1,)))
NPARAMS = sum(int(np.prod(s)) for _, s in PARAM_SHAPES)


def splitmix64(seed: int, keys) -> np.ndarray:
    """Draws ``keys`` (uint64 array) of the SplitMix64 stream seeded with
    ``seed``: z = seed + (key + 1) * golden, then the two xor-shift-multiply
    rounds and the final xor-shift of SplitMix64 (Steele, Lea, Flood,
    OOPSLA 2014)."""
    k = np.asarray(keys, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & M64) + (k + np.uint64(1)) * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def unit(r: np.ndarray) -> np.ndarray:
    """u in [0, 1) from the top 53 bits of a draw (exact in FP64)."""
    return (r >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def walk_key(w, t, j):
    """Draw index of walker w, step t (1-based), purpose j."""
    return (np.asarray(w, dtype=np.uint64) * np.uint64(STEPS) + np.uint64(t - 1)) * np.uint64(4) + np.uint64(j)


def walk_counts(g, seeds, walkers: int, damping: float, seed: int, steps: int = STEPS) -> np.ndarray:
    """counts[t-1, v] = walkers at v after step t (int64, steps x n)."""
    S = np.asarray(seeds, dtype=np.int64)
    rowptr = np.asarray(g.rowptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    outdeg = np.diff(rowptr)
    w = np.arange(walkers, dtype=np.uint64)
    pos = S[np.arange(walkers) % len(S)]
    counts = np.zeros((steps, g.n), dtype=np.int64)
    for t in range(1, steps + 1):
        u = unit(splitmix64(seed, walk_key(w, t, 0)))
        r_restart = splitmix64(seed, walk_key(w, t, 1))
        r_move = splitmix64(seed, walk_key(w, t, 2))
        d = outdeg[pos]
        restart = (u < 1.0 - damping) | (d == 0)
        nxt = np.empty_like(pos)
        nxt[restart] = S[(r_restart[restart] % np.uint64(len(S))).astype(np.int64)]
        mv = ~restart
        nxt[mv] = col[rowptr[pos[mv]] + (r_move[mv] % d[mv].astype(np.uint64)).astype(np.int64)]
        pos = nxt
        counts[t - 1] = np.bincount(pos, minlength=g.n)
    return counts


def degrees(g):
    """(indeg, outdeg) as int64 arrays."""
    outdeg = np.diff(np.asarray(g.rowptr, dtype=np.int64))
    indeg = np.diff(np.asarray(g.rowptrT, dtype=np.int64))
    return indeg, outdeg


def features(g, seeds, walkers: int, damping: float, seed: int) -> np.ndarray:
    """n x 11 feature matrix (FP64)."""
    indeg, outdeg = degrees(g)
    c = walk_counts(g, seeds, walkers, damping, seed)
    X = np.zeros((g.n, NF), dtype=np.float64)
    X[np.asarray(seeds, dtype=np.int64), 0] = 1.0
    X[:, 1] = np.log1p(indeg)
    X[:, 2] = np.log1p(outdeg)
    X[:, 3:] = np.log1p(g.n * c.T.astype(np.float64) / walkers)
    return X


def mean_in(g, Y: np.ndarray) -> np.ndarray:
    """Row v = mean of Y over the in-neighbours of v (0 without any); rows
    in CSR(A^T) order, each summed in column order."""
    rp = np.asarray(g.rowptrT, dtype=np.int64)
    colT = np.asarray(g.colT, dtype=np.int64)
    out = np.zeros((g.n,) + Y.shape[1:], dtype=np.float64)
    for v in range(g.n):
        lo, hi = rp[v], rp[v + 1]
        if hi > lo:
            out[v] = Y[colT[lo:hi]].sum(axis=0) / (hi - lo)
    return out


def unpack(theta: np.ndarray) -> dict:
    """Parameter dict from the flat vector (order of PARAM_SHAPES)."""
    p, o = {}, 0
    for name, shape in PARAM_SHAPES:
        k = int(np.prod(shape))
        p[name] = np.asarray(theta[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return p


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in PARAM_SHAPES])


def init_params(seed: int) -> np.ndarray:
    """Glorot-uniform weights, zero biases (numpy generator: a test input,
    not part of the method)."""
    rng = np.random.default_rng(seed)
    lim1 = np.sqrt(6.0 / (NF + HID))
    lim2 = np.sqrt(6.0 / (HID + 1))
    p = {"W1s": rng.uniform(-lim1, lim1, (HID, NF)), "W1n": rng.uniform(-lim1, lim1, (HID, NF)),
         "b1": np.zeros(HID), "w2s": rng.uniform(-lim2, lim2, HID), "w2n": rng.uniform(-lim2, lim2, HID),
         "b2": np.zeros(1)}
    return pack(p)


def forward(g, theta: np.ndarray, X: np.ndarray) -> dict:
    """All intermediate values of the two layers."""
    p = unpack(theta)
    M = mean_in(g, X)
    pre = X @ p["W1s"].T + M @ p["W1n"].T + p["b1"]
    H = np.maximum(pre, 0.0)
    a = H @ p["w2s"] + p["b2"][0]
    q = H @ p["w2n"]
    z = a + mean_in(g, q)
    return {"M": M, "pre": pre, "H": H, "a": a, "q": q, "z": z}


def z_at(g, theta: np.ndarray, feat, vertices) -> np.ndarray:
    """z of the given vertices only, each computed from its two-hop
    in-neighbourhood (for spot checks on graphs too large for ``forward``).
    ``feat(u)`` returns the 11 features of vertex u."""
    p = unpack(theta)
    rp = np.asarray(g.rowptrT, dtype=np.int64)
    colT = np.asarray(g.colT, dtype=np.int64)

    def mean_feat(u):
        nb = colT[rp[u]:rp[u + 1]]
        if len(nb) == 0:
            return np.zeros(NF)
        return np.sum([feat(int(w)) for w in nb], axis=0) / len(nb)

    def hidden(u):
        pre = p["W1s"] @ feat(u) + p["W1n"] @ mean_feat(u) + p["b1"]
        return np.maximum(pre, 0.0)

    out = np.empty(len(vertices))
    for i, v in enumerate(vertices):
        a = hidden(v) @ p["w2s"] + p["b2"][0]
        nb = colT[rp[v]:rp[v + 1]]
        mq = np.mean([hidden(int(u)) @ p["w2n"] for u in nb]) if len(nb) else 0.0
        out[i] = a + mq
    return out


def softmax(z: np.ndarray) -> np.ndarray:
    e = np.exp(z - z.max())
    return e / e.sum()


def kl_loss(x_star: np.ndarray, x0: np.ndarray) -> float:
    """KL(x* || x0); terms with x*_v = 0 contribute nothing."""
    nz = x_star > 0
    return float(np.sum(x_star[nz] * (np.log(x_star[nz]) - np.log(x0[nz]))))


def backward(g, theta: np.ndarray, X: np.ndarray, x_star: np.ndarray):
    """(loss, flat gradient) of KL(x* || softmax(z(theta)))."""
    p = unpack(theta)
    f = forward(g, theta, X)
    x0 = softmax(f["z"])
    loss = kl_loss(x_star, x0)
    gz = x0 - x_star
    indeg, _ = degrees(g)
    # z_v = a_v + mean over in(v) of q_u: q_u feeds every out-neighbour v of u
    # with weight 1 / indeg_v
    t = np.where(indeg > 0, gz / np.maximum(indeg, 1), 0.0)
    rp = np.asarray(g.rowptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    gq = np.zeros(g.n)
    for u in range(g.n):
        gq[u] = t[col[rp[u]:rp[u + 1]]].sum()
    ga = gz
    gH = np.outer(ga, p["w2s"]) + np.outer(gq, p["w2n"])
    gpre = gH * (f["pre"] > 0)
    grads = {"W1s": gpre.T @ X, "W1n": gpre.T @ f["M"], "b1": gpre.sum(axis=0),
             "w2s": f["H"].T @ ga, "w2n": f["H"].T @ gq, "b2": np.array([ga.sum()])}
    return loss, pack(grads)


def adam_step(theta, grad, m, v, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step t >= 1); returns (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def predict_x0(g, theta, seeds, walkers, damping, seed):
    """Warm start: softmax of the network output, or the teleport vector if
    that is not a finite positive distribution."""
    X = features(g, seeds, walkers, damping, seed)
    z = forward(g, theta, X)["z"]
    if not np.all(np.isfinite(z)):
        x0 = None
    else:
        x0 = softmax(z)
        if not (np.all(np.isfinite(x0)) and x0.sum() > 0):
            x0 = None
    if x0 is None:
        v = np.zeros(g.n)
        v[np.asarray(seeds)] = 1.0 / len(seeds)
        return v, True
    return x0, False
