"""Pins of the oracle's per-trial matrix (batched-trials reading).

One channel sampling pass draws every sample's length r from a distribution
pi and keeps r beside the column; trial t then estimates its own counts as
sum_r (s_r / pi_r) W_r and applies Eq. (1) (section 4.4: many trials of the
length weights s share one graph; section 3 and Eq. (1) for the matrix).
These tests fix ``oracle.trial_matrix`` by two routes that do not go through
its own arithmetic:

* with the trial's s equal to the pass's pi every coefficient is 1, so the
  mixture is the plain count matrix and the result must be the plain
  sparsified NetMF matrix of the same samples (``oracle.netmf_sparse``, whose
  keep decision is an exact 128-bit integer test);
* a channel matrix written out by hand on the kite graph, with the expected
  entries worked out as fractions below.
"""
import math

import numpy as np
import pytest

import oracle
from tests import graphs_small as gs

F = 1 << 16


def _drop_zeros(A):
    A = A.tocsr(copy=True)
    A.eliminate_zeros()
    A.sort_indices()
    return A


@pytest.mark.parametrize("case", [
    dict(T=3, pi=[0.2, 0.3, 0.5], M_per_m=200, C=0.9),
    dict(T=4, pi=[0.25, 0.25, 0.25, 0.25], M_per_m=120, C=None),
    dict(T=5, pi=[0.3, 0.7, 0.0, 0.0, 0.0], M_per_m=300, C=1.3),
])
def test_trial_with_s_equal_pi_is_the_plain_matrix(case):
    """s = pi: sum_r W_r is the plain pass's count matrix (same Philox stream,
    same samples), so trial_matrix must reproduce netmf_sparse: the same kept
    structure and ln x to a few ulps (the mixture forms x in FP64 while the
    plain path decides x > 1 exactly; an entry may differ only if its x lies
    within a few ulps of 1)."""
    from synth import sbm
    g = sbm([25, 25, 30], 0.25, 0.03, seed=4)
    p = gs.params(T=case["T"], s=case["pi"], M_per_m=case["M_per_m"], C=case["C"], m=g.m,
                  seed=17)
    R, Cext, W, _, _ = oracle.count_csr(g, p, channels=True)
    assert np.any((Cext & 15) > 0), "the pass must populate more than one length"
    A = _drop_zeros(oracle.trial_matrix(g, p, R, Cext, W, case["pi"]))
    B = _drop_zeros(oracle.netmf_sparse(g, p))
    # x for every counted pair, to recognise entries whose x sits at 1
    Rp, Cp, Wp, _, _ = oracle.count_csr(g, p)
    deg = oracle.degrees(g).astype(np.float64)
    rows = np.repeat(np.arange(g.n), np.diff(Rp))
    x = g.n_arcs ** 2 / (2.0 * p["b"] * p["M"]) * (Wp / F) / (deg[rows] * deg[Cp])
    near_one = set(zip(rows[np.abs(x - 1) < 8e-16].tolist(), Cp[np.abs(x - 1) < 8e-16].tolist()))
    ka = set(zip(*A.nonzero()))
    kb = set(zip(*B.nonzero()))
    assert ka ^ kb <= near_one, sorted(ka ^ kb)[:5]
    assert len(kb) > 100
    common = sorted(ka & kb)
    ia, ja = zip(*common)
    va = np.asarray(A[ia, ja]).ravel()
    vb = np.asarray(B[ia, ja]).ravel()
    np.testing.assert_allclose(va, vb, rtol=1e-14, atol=4e-16)


def _kite_channels():
    """A channel CSR on the kite graph (degrees 2, 3, 3, 3, 3, 2, 2; vol 18)
    with T = 2, written out by hand.  Column words are b << 4 | (r - 1);
    weights are in 2^-16 units."""
    # (row, col, r, count)
    ent = [(0, 1, 1, 6), (0, 1, 2, 3), (0, 3, 2, 12),
           (4, 6, 1, 1),
           (5, 5, 1, 2),
           (6, 4, 2, 9)]
    n = 7
    R = np.zeros(n + 1, np.int64)
    for a, _, _, _ in ent:
        R[a + 1] += 1
    R = np.cumsum(R)
    Cext = np.array([(b << 4) | (r - 1) for _, b, r, _ in ent], np.int32)
    W = np.array([c * F for _, _, _, c in ent], np.uint64)
    return R, Cext, W


def test_trial_matrix_hand_computed_two_lengths():
    """pi = (1/4, 3/4), trial s = (3/5, 2/5): coefficients s_r / pi_r =
    (12/5, 8/15).  With b = 1 and M = 162 the scale vol^2 / (2bM) is
    324 / 324 = 1, so x_ab = (sum_r coef_r c_r) / (d_a d_b) with c_r the
    count in units of 2^-16:
      (0,1): (12/5 * 6 + 8/15 * 3) / (2 * 3) = 16/6 = 8/3  -> ln(8/3)
      (0,3): (8/15 * 12) / (2 * 3)          = 16/15       -> ln(16/15)
      (5,5): (12/5 * 2) / (2 * 2)           = 6/5         -> ln(6/5)
      (4,6): (12/5 * 1) / (3 * 2)           = 2/5         -> dropped
      (6,4): (8/15 * 9) / (2 * 3)           = 4/5         -> dropped
    A dropped channel, a wrong split of the column word, a missing 2^-16 or
    a wrong volume factor each changes one of these."""
    g = gs.kite()
    assert list(np.diff(g.rowptr)) == [2, 3, 3, 3, 3, 2, 2] and g.n_arcs == 18
    R, Cext, W = _kite_channels()
    p = gs.params(T=2, s=[0.25, 0.75], M_per_m=18, m=g.m, b=1)
    assert p["M"] == 162
    A = oracle.trial_matrix(g, p, R, Cext, W, [0.6, 0.4]).toarray()
    want = np.zeros((7, 7))
    want[0, 1] = math.log(8 / 3)
    want[0, 3] = math.log(16 / 15)
    want[5, 5] = math.log(6 / 5)
    np.testing.assert_allclose(A, want, rtol=1e-14, atol=1e-15)
    # the structure carries the dropped pairs as explicit zeros
    S = oracle.trial_matrix(g, p, R, Cext, W, [0.6, 0.4])
    assert S.nnz == 5 and S[4, 6] == 0 and S[6, 4] == 0


def test_trial_matrix_rejects_unsampled_length():
    """A trial that puts weight on a length the pass never draws has no
    unbiased estimate (pi_r = 0 where s_r > 0) and is refused."""
    g = gs.kite()
    R, Cext, W = _kite_channels()
    p = gs.params(T=2, s=[1.0, 0.0], M_per_m=18, m=g.m)
    with pytest.raises(ValueError):
        oracle.trial_matrix(g, p, R, Cext, W, [0.5, 0.5])
