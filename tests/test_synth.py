"""Generators produce simple symmetric graphs of the stated shape."""
import numpy as np
import scipy.stats

from synth import chung_lu, sbm, workload


def _check_simple(g):
    deg = np.diff(g.rowptr)
    rows = np.repeat(np.arange(g.n), deg)
    assert np.all(rows != g.col)
    key = rows.astype(np.int64) * g.n + g.col
    assert np.all(np.diff(key) > 0)           # sorted, no duplicates
    rev = g.col.astype(np.int64) * g.n + rows
    assert np.array_equal(np.sort(rev), key)  # symmetric


def test_sbm_exact_law():
    g = sbm([50] * 4, 0.3, 0.02, seed=1)
    _check_simple(g)
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    same = (rows // 50) == (g.col // 50)
    m_in, m_out = same.sum() // 2, (~same).sum() // 2
    n_in, n_out = 4 * 50 * 49 // 2, 6 * 50 * 50
    assert abs(m_in - 0.3 * n_in) < 6 * np.sqrt(n_in * 0.3 * 0.7)
    assert abs(m_out - 0.02 * n_out) < 6 * np.sqrt(n_out * 0.02 * 0.98)
    assert g.labels.sum() == g.n


def test_sbm_deterministic():
    a = sbm([30] * 3, 0.2, 0.05, seed=4)
    b = sbm([30] * 3, 0.2, 0.05, seed=4)
    assert np.array_equal(a.col, b.col) and np.array_equal(a.rowptr, b.rowptr)


def test_chung_lu_exact_m_and_power_law():
    g = chung_lu(5000, 40000, 2.2, seed=3)
    _check_simple(g)
    assert g.m == 40000
    deg = np.diff(g.rowptr)
    # heavy tail: the largest degree is far above the mean
    assert deg.max() > 10 * deg.mean()
    # tail exponent of the degree sequence is near gamma (rough MLE, x_min = 10)
    x = deg[deg >= 10].astype(float)
    alpha = 1 + len(x) / np.sum(np.log(x / 9.5))
    assert 1.8 < alpha < 2.8


def test_chung_lu_groups():
    g = chung_lu(2000, 20000, 2.2, seed=5, n_groups=7)
    _check_simple(g)
    k = g.labels.sum(1)
    assert k.min() >= 1 and k.max() <= 3
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    shared = np.any(g.labels[rows] & g.labels[g.col], axis=1).mean()
    assert shared > 0.6


def test_tiny_workload_matches_configuration():
    g, p = workload("tiny")
    assert g.n == 1000 and abs(g.m - 9675) < 6 * 90
    assert p["M"] == 100 * 10 * g.m and p["d"] == 32 and p["q"] == 1


def test_relabel_is_an_isomorphism():
    from synth import relabel
    from tests import graphs_small as gs
    g = gs.with_weights(workload("tiny")[0], 4)
    h = relabel(g, 7)
    assert h.n == g.n and h.n_arcs == g.n_arcs
    # the permutation drawn from the same seed carries the weighted arcs of
    # g exactly onto those of h
    import torch
    perm = torch.randperm(g.n, generator=torch.Generator().manual_seed(7)).numpy()
    arcs = lambda gr: {(int(u), int(v), int(w)) for u in range(gr.n)
                       for v, w in zip(gr.col[gr.rowptr[u]:gr.rowptr[u + 1]],
                                       gr.weight[gr.rowptr[u]:gr.rowptr[u + 1]])}
    assert {(perm[u], perm[v], w) for u, v, w in arcs(g)} == arcs(h)
    for u in range(h.n):
        assert np.all(np.diff(h.col[h.rowptr[u]:h.rowptr[u + 1]]) > 0)
    assert np.array_equal(h.labels[perm], g.labels)
