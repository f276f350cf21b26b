"""Seeded held-out edges and corrupted edges for link-prediction evaluation.

The protocol of the paper's very-large-graph runs (after PyTorch-BigGraph):
a random set of edges is removed from the training graph, and each removed
edge (u, v) is later ranked against K corrupted edges (u, w) with w drawn
uniformly from the vertices other than v.  Pure functions of their seeds; no
part of the embedding method.
"""
from __future__ import annotations

import numpy as np

from .graphs import Graph


def holdout_edges(g: Graph, count: int, seed: int):
    """Removes `count` distinct undirected edges, drawn uniformly, from g.

    Returns (train graph, pos) with pos an int32 (count x 2) array of the
    removed edges, each oriented at random ((u, v) or (v, u))."""
    rng = np.random.default_rng(seed)
    rowptr = np.asarray(g.rowptr, dtype=np.int64)
    col = np.asarray(g.col)
    n_arcs = int(rowptr[-1])
    m = n_arcs // 2
    if not 0 < count <= m:
        raise ValueError("count must be in [1, m]")
    # an undirected edge is its single arc with u < v: draw arcs uniformly and
    # keep the upward ones until `count` distinct edges are found
    chosen = np.empty(0, dtype=np.int64)
    while len(chosen) < count:
        arcs = rng.integers(0, n_arcs, size=4 * (count - len(chosen)) + 64)
        rows = np.searchsorted(rowptr, arcs, side="right") - 1
        up = arcs[col[arcs] > rows]
        chosen = np.unique(np.concatenate([chosen, up]))
        if len(chosen) > count:
            chosen = rng.permutation(chosen)[:count]
            chosen.sort()
    u = np.searchsorted(rowptr, chosen, side="right") - 1
    v = col[chosen].astype(np.int64)
    # the reverse arcs (v, u)
    rev = np.empty(count, dtype=np.int64)
    for i in range(count):
        b, e = rowptr[v[i]], rowptr[v[i] + 1]
        rev[i] = b + np.searchsorted(col[b:e], u[i])
    assert np.all(col[rev] == u)
    drop = np.concatenate([chosen, rev])
    keep = np.ones(n_arcs, dtype=bool)
    keep[drop] = False
    removed = np.bincount(np.concatenate([u, v]), minlength=g.n)
    deg = np.diff(rowptr) - removed
    new_rowptr = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(deg, out=new_rowptr[1:])
    train = Graph(g.n, new_rowptr, col[keep], g.labels, g.name + "-train")
    flip = rng.random(count) < 0.5
    a = np.where(flip, v, u)
    b = np.where(flip, u, v)
    return train, np.stack([a, b], axis=1).astype(np.int32)


def corrupt_destinations(pos, n: int, K: int, seed: int):
    """int32 (len(pos) x K) array of corrupted destinations: uniform over the
    vertices other than each edge's own destination."""
    rng = np.random.default_rng(seed)
    pos = np.asarray(pos)
    w = rng.integers(0, n - 1, size=(len(pos), K))
    w += (w >= pos[:, 1:2]).astype(w.dtype)
    return w.astype(np.int32)
