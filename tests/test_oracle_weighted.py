"""Pins of the oracle's weighted-graph sampler (positive integer weights A_uv,
degree sampling p_e = min(1, C A_uv (1/d_u + 1/d_v)), walk steps with
probability A_xy / d_x, sample weight h / p_e with h = r / sum_j 1/A_j over
the path's r edges).

The path factor is what makes the estimator exact: for a path x_0..x_r whose
centre edge is j, the sampler emits it with probability
(1/r) prod_{i != j} A_i / prod_{0<i<r} d_{x_i} (per sample of edge j), so
summing h times that over the r possible centres gives
prod_i A_i / prod_{0<i<r} d_{x_i}, the path's term of A (D^-1 A)^(r-1):
    E[W] = 2^F (M/m) sum_r s_r A (D^-1 A)^(r-1)
exactly as for unweighted graphs (where h = 1).  The brute-force test checks
this derivation without the oracle; the others check the oracle against it.
"""
import numpy as np
import pytest

import oracle
from tests import graphs_small as gs

F = 2 ** 16


def expected_W(g, s, M):
    A = gs.dense_wadj(g)
    P = A / A.sum(1, keepdims=True)
    E = np.zeros_like(A)
    Pk = np.eye(g.n)
    for r in range(1, len(s) + 1):
        E += s[r - 1] * (A @ Pk)
        Pk = Pk @ P
    return F * (M / g.m) * E


def dense_counts(g, R, C, W):
    out = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(R))
    out[rows, C] = W.astype(np.float64)
    return out


def test_path_factor_makes_the_estimator_exact():
    """Brute force over every edge, length, split and weighted neighbour
    choice of tiny weighted graphs: sum of probability x h per pair equals
    the closed form."""
    for g in (gs.with_weights(gs.kite(), 1), gs.with_weights(gs.star(5), 2),
              gs.with_weights(gs.path(5), 3)):
        s = [0.2, 0.5, 0.3]
        A = gs.dense_wadj(g)
        deg = A.sum(1)
        nb = [g.col[g.rowptr[i]:g.rowptr[i + 1]] for i in range(g.n)]
        E = np.zeros((g.n, g.n))

        def walks(x, steps):
            """(end vertex, probability, sum of 1/A over the steps)."""
            if steps == 0:
                yield x, 1.0, 0.0
                return
            for y in nb[x]:
                for z, p, inv in walks(int(y), steps - 1):
                    yield z, p * A[x, y] / deg[x], inv + 1.0 / A[x, y]

        for u in range(g.n):
            for v in nb[u]:
                if v <= u:
                    continue
                for r in range(1, 4):
                    for j in range(r):
                        for a, pa, ia in walks(u, j):
                            for b, pb, ib in walks(int(v), r - 1 - j):
                                h = r / (1.0 / A[u, v] + ia + ib)
                                pr = s[r - 1] / r * pa * pb * h
                                E[a, b] += pr
                                E[b, a] += pr
        M = 7 * g.m
        np.testing.assert_allclose(F * (M / g.m) * E, expected_W(g, s, M), rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("C", [None, 0.8])
def test_unit_weights_are_the_unweighted_sampler(C):
    """Weights all 1: every slot, count and Eq. (1) entry is bit-identical to
    the unweighted oracle."""
    g = gs.kite()
    g1 = gs.Graph(g.n, g.rowptr, g.col, None, "kite-1", np.ones(g.n_arcs, np.uint32))
    p = gs.params(T=3, s=[0.2, 0.5, 0.3], M_per_m=50, C=C, m=g.m, seed=9)
    a, b = oracle.sample_slots(g, p), oracle.sample_slots(g1, p)
    for key in a:
        np.testing.assert_array_equal(a[key], b[key])
    R0, C0, W0, t0, c0 = oracle.count_csr(g, p)
    R1, C1, W1, t1, c1 = oracle.count_csr(g1, p)
    for x, y in ((R0, R1), (C0, C1), (W0, W1)):
        np.testing.assert_array_equal(x, y)
    assert (t0, c0) == (t1, c1)
    k0, v0 = oracle.trunc_log(g, p, R0, C0, W0)
    k1, v1 = oracle.trunc_log(g1, p, R1, C1, W1)
    np.testing.assert_array_equal(k0, k1)
    np.testing.assert_array_equal(v0, v1)


def test_weighted_line_case_is_exact():
    """T = 1, no downsampling, integer M/m: W = (M/m) 2^F A exactly (h = A_uv
    for a one-edge path) and the truncated log is the weighted LINE matrix
    log(vol A_ab / (b d_a d_b))."""
    for g, b in ((gs.with_weights(gs.kite(), 4), 1), (gs.with_weights(gs.complete(5), 5), 2)):
        p = gs.params(T=1, s=[1.0], M_per_m=3, C=None, m=g.m, b=b)
        R, C, W, att, acc = oracle.count_csr(g, p)
        A = gs.dense_wadj(g)
        np.testing.assert_array_equal(dense_counts(g, R, C, W), 3 * F * A)
        keep, val = oracle.trunc_log(g, p, R, C, W)
        deg = A.sum(1)
        vol = deg.sum()
        rows = np.repeat(np.arange(g.n), np.diff(R))
        x = vol * A[rows, C] / (b * deg[rows] * deg[C])
        np.testing.assert_array_equal(keep, x > 1)
        np.testing.assert_allclose(val[keep], np.log(x[keep]), rtol=0, atol=4e-16)


@pytest.mark.parametrize("C", [None, 0.5])
def test_weighted_expected_counts_z_scores(C):
    """The oracle's counts on a weighted graph follow the closed form, with
    and without degree downsampling (importance weights keep it unbiased)."""
    g = gs.with_weights(gs.kite(), 6)
    s = [0.2, 0.5, 0.3]
    p = gs.params(T=3, s=s, M_per_m=20000, C=C, m=g.m, seed=3)
    R, Cc, W, att, acc = oracle.count_csr(g, p, nthreads=3)
    obs = dense_counts(g, R, Cc, W)
    np.testing.assert_array_equal(obs, obs.T)
    exp = expected_W(g, s, p["M"])
    A = gs.dense_wadj(g)
    deg = A.sum(1)
    # largest single-sample weight: h <= r max A, over p_e
    pmin = 1.0 if C is None else min(1.0, min(C * A[u, v] * (1 / deg[u] + 1 / deg[v])
                                              for u in range(g.n) for v in range(g.n) if A[u, v]))
    wmax = F * 3 * A.max() / pmin
    z = np.abs(obs - exp) / np.sqrt(2 * wmax * exp + 1e-9)
    assert z.max() < 6, z.max()
    assert np.all(obs[exp == 0] == 0)


def test_weighted_degrees_and_volume():
    g = gs.with_weights(gs.kite(), 7)
    A = gs.dense_wadj(g)
    np.testing.assert_array_equal(oracle.degrees(g), A.sum(1).astype(np.int64))
    assert oracle.volume(g) == int(A.sum())


def test_zero_weight_is_rejected():
    g = gs.with_weights(gs.kite(), 8)
    w = g.weight.copy()
    w[3] = 0
    bad = gs.Graph(g.n, g.rowptr, g.col, None, "bad", w)
    with pytest.raises(ValueError):
        oracle.count_csr(bad, gs.params(m=g.m))
