"""Hand-built tiny graphs for closed-form checks."""
import numpy as np

from synth import Graph


def from_edges(n, edges, name=""):
    a = np.array([min(e) for e in edges] + [max(e) for e in edges], dtype=np.int64)
    b = np.array([max(e) for e in edges] + [min(e) for e in edges], dtype=np.int64)
    order = np.lexsort((b, a))
    a, b = a[order], b[order]
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, a + 1, 1)
    return Graph(n, np.cumsum(rowptr), b.astype(np.int32), None, name)


def kite():
    """7 vertices, irregular degrees, triangles and a pendant path."""
    return from_edges(7, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3), (3, 4), (4, 5),
                          (4, 6), (5, 6)], "kite")


def path(n):
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], f"path{n}")


def star(n):
    return from_edges(n, [(0, i) for i in range(1, n)], f"star{n}")


def cycle(n):
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], f"cycle{n}")


def complete(n):
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)], f"K{n}")


def dense_adj(g):
    A = np.zeros((g.n, g.n))
    r = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    A[r, g.col] = 1.0
    return A


def params(T=3, s=None, M_per_m=10, C=None, seed=1, m=1, **kw):
    s = np.full(T, 1.0 / T) if s is None else np.asarray(s, float)
    p = dict(T=T, s=s, M=int(M_per_m * m), b=1, C=C, seed=seed, d=2, oversample=2,
             q=1, cheb_k=5, theta=0.5, mu=0.2, precision="f64")
    p.update(kw)
    return p


def with_weights(g, seed, wmax=9):
    """g with symmetric positive integer arc weights drawn from 1..wmax."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    lo = np.minimum(rows, g.col)
    hi = np.maximum(rows, g.col)
    key = lo.astype(np.int64) * g.n + hi
    uniq, inv = np.unique(key, return_inverse=True)
    w = rng.integers(1, wmax + 1, size=len(uniq)).astype(np.uint32)[inv]
    return Graph(g.n, g.rowptr, g.col, g.labels, g.name + "-w", w)


def dense_wadj(g):
    A = np.zeros((g.n, g.n))
    r = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    A[r, g.col] = 1.0 if g.weight is None else g.weight.astype(np.float64)
    return A
