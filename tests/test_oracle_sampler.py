"""Pins of the oracle's sparsifier (section 5.2 and the two sampling
algorithms) against closed forms and invariants that need no implementation.

Law used throughout (derived from the PathSampling algorithm): for an edge
(u, v), length r and uniform split j, the emitted ordered pair is distributed
as (1/r) sum_j P^j[u, a] P^(r-1-j)[v, b] with P = D^-1 A.  Summed over both
orientations of every edge this gives
    E[W] = 2^F (M/m) sum_r s_r A P^(r-1)
(the brute-force test below checks this derivation by enumerating walks), and
Eq. (1) is recovered as vol^2/(2bM) W/(d_a d_b) -> vol/b sum_r s_r P^r D^-1.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.stats

import oracle
from tests import graphs_small as gs

F = 2 ** 16


def walk_matrix(g):
    A = gs.dense_adj(g)
    return A, A / A.sum(1, keepdims=True)


def expected_W(g, s, M):
    A, P = walk_matrix(g)
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


# ---------------------------------------------------------------------------
def test_closed_form_matches_walk_enumeration():
    """Brute force: enumerate every edge, length, split and neighbour choice
    of tiny graphs and sum exact path probabilities."""
    for g in (gs.kite(), gs.path(4), gs.star(4)):
        s = [0.2, 0.5, 0.3]
        deg = g.degrees()
        nb = [g.col[g.rowptr[i]:g.rowptr[i + 1]] for i in range(g.n)]
        E = np.zeros((g.n, g.n))

        def walks(x, steps):
            if steps == 0:
                yield x, 1.0
                return
            for y in nb[x]:
                for z, p in walks(int(y), steps - 1):
                    yield z, p / deg[x]

        for u in range(g.n):
            for v in nb[u]:
                if v <= u:
                    continue
                for r in range(1, 4):
                    for j in range(r):
                        for a, pa in walks(u, j):
                            for b, pb in walks(int(v), r - 1 - j):
                                pr = s[r - 1] / r * pa * pb
                                E[a, b] += pr
                                E[b, a] += pr
        M = 7 * g.m
        np.testing.assert_allclose(F * (M / g.m) * E, expected_W(g, s, M), rtol=1e-12, atol=1e-9)


def test_line_case_is_exact():
    """T = 1, no downsampling, integer M/m: W = (M/m) 2^F A exactly and the
    truncated log equals the LINE matrix log(vol / (b d_a d_b))."""
    for g, b in ((gs.kite(), 1), (gs.kite(), 2), (gs.complete(5), 1)):
        p = gs.params(T=1, s=[1.0], M_per_m=3, C=None, m=g.m, b=b)
        R, C, W, att, acc = oracle.count_csr(g, p)
        A = gs.dense_adj(g)
        np.testing.assert_array_equal(dense_counts(g, R, C, W), 3 * F * A)
        keep, val = oracle.trunc_log(g, p, R, C, W)
        deg = g.degrees()
        rows = np.repeat(np.arange(g.n), np.diff(R))
        x = g.n_arcs / (b * deg[rows] * deg[C])
        np.testing.assert_array_equal(keep, x > 1)
        np.testing.assert_allclose(val[keep], np.log(x[keep]), rtol=0, atol=4e-16)
        assert att == acc == 3 * g.m


def test_trunc_log_boundary_is_strict():
    """x = 1 exactly is dropped (K_{4,4}, b = 2: vol = 32 = b d_a d_b)."""
    k44 = gs.from_edges(8, [(i, j) for i in range(4) for j in range(4, 8)])
    p = gs.params(T=1, s=[1.0], M_per_m=5, C=None, m=k44.m, b=2)
    R, C, W, _, _ = oracle.count_csr(k44, p)
    keep, _ = oracle.trunc_log(k44, p, R, C, W)
    assert len(W) == 32 and not keep.any()
    # one unit of weight either side of the boundary
    deg = k44.degrees()
    Wp = W.copy()
    Wp[0] += 1
    Wm = W.copy()
    Wm[1] -= 1
    kp, _ = oracle.trunc_log(k44, p, R, C, Wp)
    km, _ = oracle.trunc_log(k44, p, R, C, Wm)
    assert kp[0] and not km[1]
    assert deg[0] == 4


def test_per_edge_law_chi_square():
    """For one edge, the empirical law of (r, u', v') over many samples
    matches s_r (1/r) sum_j P^j[u, .] P^(r-1-j)[v, .]."""
    g = gs.kite()
    _, P = walk_matrix(g)
    s = np.array([0.2, 0.5, 0.3])
    p = gs.params(T=3, s=s, M_per_m=40000, C=None, m=g.m, seed=11)
    for e in (0, 3, 6):
        out = oracle.sample_slots(g, p, e, e + 1)
        u, v = None, None
        # edge e in CSR order of (u < v) arcs
        k = 0
        for uu in range(g.n):
            for vv in g.col[g.rowptr[uu]:g.rowptr[uu + 1]]:
                if vv > uu:
                    if k == e:
                        u, v = uu, int(vv)
                    k += 1
        assert out["acc"].all()
        obs = np.zeros((3, g.n, g.n))
        np.add.at(obs, (out["r"].astype(int) - 1, out["a"], out["b"]), 1)
        exp = np.zeros_like(obs)
        for r in range(1, 4):
            for j in range(r):
                exp[r - 1] += s[r - 1] / r * np.outer(np.linalg.matrix_power(P, j)[u],
                                                       np.linalg.matrix_power(P, r - 1 - j)[v])
        exp *= len(out["r"])
        mask = exp > 5
        assert obs[~mask].sum() <= max(50, 3 * exp[~mask].sum())
        o = obs[mask]
        x = exp[mask]
        stat = scipy.stats.chisquare(o, x * o.sum() / x.sum())
        assert stat.pvalue > 1e-6, (e, stat)


@pytest.mark.parametrize("C", [None, 0.5])
def test_expected_counts_z_scores(C):
    """E[W] = 2^F (M/m) sum_r s_r A P^(r-1), with and without degree
    downsampling (downsampling keeps the estimator unbiased, Theorem 1)."""
    g = gs.kite()
    s = [0.2, 0.5, 0.3]
    p = gs.params(T=3, s=s, M_per_m=20000, C=C, m=g.m, seed=3)
    R, Cc, W, att, acc = oracle.count_csr(g, p, nthreads=3)
    obs = dense_counts(g, R, Cc, W)
    np.testing.assert_array_equal(obs, obs.T)
    exp = expected_W(g, s, p["M"])
    if C is None:
        wmax = F
        assert acc == att
    else:
        deg = g.degrees()
        wmax = max(round(F / (C * (1 / deg[u] + 1 / deg[v])))
                   for u in range(g.n) for v in g.col[g.rowptr[u]:g.rowptr[u + 1]])
    z = np.abs(obs - exp) / np.sqrt(2 * wmax * exp + 1e-9)
    assert z.max() < 6, z.max()
    # entries that cannot be reached are exactly zero
    assert np.all(obs[exp == 0] == 0)


def test_total_weight_invariants():
    """No downsampling: sum W = 2 2^F sum_e n_e exactly.  With downsampling:
    E[sum W] = sum_e n_e p_e 2 rint(2^F / p_e), which is 2 2^F M up to the
    rounding of the weights (Theorem 1)."""
    g = gs.kite()
    p = gs.params(T=3, s=[0.3, 0.3, 0.4], M_per_m=5000, C=None, m=g.m, seed=4)
    R, Cc, W, att, acc = oracle.count_csr(g, p)
    assert int(W.sum()) == 2 * F * att
    C = 0.6
    p = gs.params(T=3, s=[0.3, 0.3, 0.4], M_per_m=5000, C=C, m=g.m, seed=4)
    R, Cc, W, att, acc = oracle.count_csr(g, p)
    deg = g.degrees()
    mean = var = exp_acc = 0.0
    ne = p["M"] // g.m
    for u in range(g.n):
        for v in g.col[g.rowptr[u]:g.rowptr[u + 1]]:
            if v <= u:
                continue
            pe = min(1.0, C * (1 / deg[u] + 1 / deg[v]))
            w = F if pe >= 1 else round(F / pe)
            mean += ne * pe * 2 * w
            var += ne * pe * (1 - pe) * (2 * w) ** 2
            exp_acc += ne * pe
    assert abs(mean - 2 * F * p["M"]) / (2 * F * p["M"]) < 1e-4
    assert abs(float(W.sum()) - mean) < 6 * math.sqrt(var)
    assert abs(acc - exp_acc) < 6 * math.sqrt(exp_acc)


def test_expected_sample_count_is_M():
    """n_e = floor(M/m) + Bernoulli(frac(M/m)) so E[sum n_e] = M."""
    g = gs.from_edges(40, [(i, j) for i in range(40) for j in range(i + 1, 40) if (i * 7 + j) % 5 == 0])
    m = g.m
    M = 3 * m + (m * 3) // 7
    f = (M / m) % 1
    tot = 0
    runs = 20
    for seed in range(runs):
        p = gs.params(T=2, s=[0.5, 0.5], M_per_m=1, C=None, m=m, seed=seed)
        p["M"] = M
        out = oracle.sample_slots(g, p)
        per_edge = np.bincount(out["e"], minlength=m)
        assert set(np.unique(per_edge)) <= {M // m, M // m + 1}
        tot += len(out["e"])
    z = abs(tot - runs * M) / math.sqrt(runs * m * f * (1 - f))
    assert z < 6


def test_row_sums_follow_degrees():
    """E[sum_b W_ab] = 2^F (M/m) d_a because P 1 = 1."""
    g = gs.kite()
    p = gs.params(T=3, s=[0.1, 0.6, 0.3], M_per_m=20000, C=None, m=g.m, seed=8)
    R, Cc, W, _, _ = oracle.count_csr(g, p)
    rs = dense_counts(g, R, Cc, W).sum(1)
    exp = F * (p["M"] / g.m) * g.degrees()
    z = np.abs(rs - exp) / np.sqrt(2 * F * exp)
    assert z.max() < 6


def test_kept_edge_bound():
    """sum_e p_e <= C n (degree sampling keeps O(n C) edges, section 4.1)."""
    from synth import workload
    g, p = workload("tiny")
    deg = g.degrees()
    rows = np.repeat(np.arange(g.n), deg)
    up = g.col > rows
    pe = np.minimum(1.0, p["C"] * (1 / deg[rows[up]] + 1 / deg[g.col[up]]))
    assert pe.sum() <= p["C"] * g.n


def test_eq1_limit():
    """With many samples the truncated log approaches Eq. (1)'s dense matrix
    trunc_log(vol/b sum_r s_r P^r D^-1) entry by entry."""
    g = gs.kite()
    s = np.array([0.2, 0.5, 0.3])
    p = gs.params(T=3, s=s, M_per_m=200000, C=None, m=g.m, seed=12)
    R, Cc, W, _, _ = oracle.count_csr(g, p)
    keep, val = oracle.trunc_log(g, p, R, Cc, W)
    A, P = walk_matrix(g)
    deg = g.degrees()
    dense = np.zeros_like(P)
    Pr = np.eye(g.n)
    for r in range(1, 4):
        Pr = Pr @ P
        dense += s[r - 1] * Pr
    dense = g.n_arcs / p["b"] * dense / deg[None, :]
    exp_counts = expected_W(g, s, p["M"]) / F
    rows = np.repeat(np.arange(g.n), np.diff(R))
    for i in range(len(Cc)):
        a, b = rows[i], Cc[i]
        x = dense[a, b]
        tol = 6 * math.sqrt(2 / exp_counts[a, b])
        if x > 1 + 2 * tol:
            assert keep[i]
            assert abs(val[i] - math.log(x)) < 2 * tol
        elif x < 1 - 2 * tol:
            assert not keep[i]


def test_row_window_and_slots_agree_with_full():
    """Internal consistency: the threaded aggregator restricted to a row
    window equals the full result's rows, and equals summing the per-slot
    enumeration."""
    from synth import sbm
    g = sbm([30, 30, 30], 0.2, 0.02, seed=2)
    p = gs.params(T=4, s=[0.1, 0.2, 0.3, 0.4], M_per_m=50, C=math.log(g.n), m=g.m, seed=6)
    R, Cc, W, att, acc = oracle.count_csr(g, p, nthreads=4)
    R2, C2, W2, att2, acc2 = oracle.count_csr(g, p, row_lo=20, row_hi=55, nthreads=2)
    lo, hi = R[20], R[55]
    np.testing.assert_array_equal(C2, Cc[lo:hi])
    np.testing.assert_array_equal(W2, W[lo:hi])
    np.testing.assert_array_equal(R2, R[20:56] - R[20])
    assert (att, acc) == (att2, acc2)
    out = oracle.sample_slots(g, p)
    dense = np.zeros((g.n, g.n), np.uint64)
    ok = out["acc"].astype(bool)
    np.add.at(dense, (out["a"][ok], out["b"][ok]), out["w"][ok])
    np.add.at(dense, (out["b"][ok], out["a"][ok]), out["w"][ok])
    np.testing.assert_array_equal(dense_counts(g, R, Cc, W).astype(np.uint64), dense)
    assert ok.sum() == acc and len(ok) == att


@pytest.mark.parametrize("pi", [[1, 1, 1], [0.2, 0.3, 0.5]])
def test_channel_mixture_is_unbiased_for_each_trial(pi):
    """Batched trials share one pass whose lengths are drawn from pi and
    weight the length-r channel by s_r / pi_r: for any s the mixture has the
    expectation E[W] = 2^F (M/m) sum_r s_r A P^(r-1) of the trial's own
    sampler."""
    g = gs.kite()
    T = 3
    p = gs.params(T=T, s=pi, M_per_m=30000, C=0.5, m=g.m, seed=21)
    pi = np.asarray(pi, float) / np.sum(pi)
    R, Cext, W, att, acc = oracle.count_csr(g, p, channels=True)
    rows = np.repeat(np.arange(g.n), np.diff(R))
    chan = np.zeros((T, g.n, g.n))
    np.add.at(chan, (Cext & 15, rows, Cext >> 4), W.astype(np.float64))
    # each channel holds the samples of its length only, in proportion pi_r
    per = np.array([chan[r].sum() for r in range(T)])
    assert np.allclose(per / per.sum(), pi, atol=0.02)
    deg = g.degrees()
    wmax = max(round(F / min(1.0, 0.5 * (1 / deg[u] + 1 / deg[v])))
               for u in range(g.n) for v in g.col[g.rowptr[u]:g.rowptr[u + 1]])
    for s in ([0.2, 0.5, 0.3], [1.0, 0.0, 0.0], [0.0, 0.1, 0.9]):
        s = np.asarray(s)
        mixed = np.tensordot(s / pi, chan, axes=1)
        exp = expected_W(g, s, p["M"])
        var = 2 * wmax * max(s / pi) * exp + 1e-9
        z = np.abs(mixed - exp) / np.sqrt(var)
        assert z.max() < 6, (s, z.max())


def test_edge_subset_reproduces_row_windows():
    """With walk lengths r <= 2 the rows of a window only receive samples of
    edges incident to the window's closed neighbourhood: the oracle run on
    those edges alone gives the window's rows exactly (the device's
    full-size parity checks rely on this)."""
    from synth import workload
    g, p = workload("tiny")
    p = dict(p, T=5, s=np.array([0.3, 0.7, 0.0, 0.0, 0.0]), M=40 * 5 * g.m, seed=9)
    ids = oracle.edge_ids(g)
    assert np.all(np.bincount(ids) == 2) and ids.max() == g.m - 1
    for lo, hi in ((0, 3), (500, 507), (g.n - 4, g.n)):
        nb = set(range(lo, hi))
        for a in range(lo, hi):
            nb.update(g.col[g.rowptr[a]:g.rowptr[a + 1]].tolist())
        arcs = np.concatenate([np.arange(g.rowptr[b], g.rowptr[b + 1]) for b in sorted(nb)])
        sel = oracle.edge_ids_of(g, arcs)
        np.testing.assert_array_equal(sel, ids[arcs])
        R0, C0, W0, _, _ = oracle.count_csr(g, p, row_lo=lo, row_hi=hi)
        R1, C1, W1 = oracle.count_csr_edges(g, p, lo, hi, sel)
        np.testing.assert_array_equal(R0, R1)
        np.testing.assert_array_equal(C0, C1)
        np.testing.assert_array_equal(W0, W1)
    Om = oracle.gaussian_omega(g.n, 9, 5)
    np.testing.assert_array_equal(oracle.gaussian_omega(g.n, 9, 5, rows=[3, 0, 999]), Om[[3, 0, 999]])
