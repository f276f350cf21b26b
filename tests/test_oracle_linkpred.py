"""The link-prediction oracle pinned to independent definitions: the
Mann-Whitney AUC of scikit-learn, scipy's tie-aware ranking, hand-computed
metrics, and the closed forms of a perfect and of a constant embedding.  Also
pins the held-out-edge generator (removed edges gone, everything else kept)."""
import numpy as np
import pytest
from scipy.stats import rankdata
from sklearn.metrics import roc_auc_score

from oracle import linkpred
from synth import workload, holdout_edges, corrupt_destinations


def _case(seed, n=300, d=8, h=40, K=25, integer=False):
    rng = np.random.default_rng(seed)
    X = rng.integers(-2, 3, size=(n, d)).astype(np.float64) if integer else rng.standard_normal((n, d))
    pos = np.stack([rng.integers(0, n, h), rng.integers(0, n, h)], axis=1)
    neg = rng.integers(0, n - 1, size=(h, K))
    neg += neg >= pos[:, 1:2]                # corrupted edges differ from the edge
    return X, pos, neg


@pytest.mark.parametrize("integer", [False, True])
def test_auc_matches_sklearn_per_edge(integer):
    X, pos, neg = _case(1, integer=integer)
    above, ties = linkpred.rank_counts(X, pos, neg)
    K = neg.shape[1]
    for i in range(len(pos)):
        sp = X[pos[i, 0]] @ X[pos[i, 1]]
        sn = X[pos[i, 0]] @ X[neg[i]].T
        y = np.r_[1, np.zeros(K)]
        ref = roc_auc_score(y, np.r_[sp, sn])
        assert abs((K - above[i] - 0.5 * ties[i]) / K - ref) < 1e-12
    if integer:
        assert ties.sum() > 0          # the integer case exercises ties


@pytest.mark.parametrize("integer", [False, True])
def test_rank_matches_scipy_rankdata(integer):
    X, pos, neg = _case(2, integer=integer)
    above, _ = linkpred.rank_counts(X, pos, neg)
    for i in range(len(pos)):
        s = np.r_[X[pos[i, 0]] @ X[pos[i, 1]], X[pos[i, 0]] @ X[neg[i]].T]
        # descending rank, ties resolved in the edge's favour
        assert 1 + above[i] == rankdata(-s, method="min")[0]


def test_metrics_hand_computed():
    above = np.array([0, 1, 4])
    ties = np.array([0, 2, 0])
    m = linkpred.metrics(above, ties, K=4, hits_k=1)
    assert m["mean_rank"] == pytest.approx(8 / 3)
    assert m["mrr"] == pytest.approx((1 + 1 / 2 + 1 / 5) / 3)
    assert m["hits"] == pytest.approx(1 / 3)
    assert m["auc"] == pytest.approx((1.0 + 0.5 + 0.0) / 3)


def test_perfect_and_constant_embeddings():
    n, K = 50, 10
    pos = np.array([[0, 1], [2, 3]])
    neg = np.tile(np.arange(10, 10 + K), (2, 1))
    X = np.zeros((n, 2))
    X[[0, 1, 2, 3], 0] = 1.0                 # the edges score 1, corrupted ones 0
    m, above, ties = linkpred.link_metrics(X, pos, neg, hits_k=1)
    assert (above == 0).all() and (ties == 0).all()
    assert m == dict(mean_rank=1.0, mrr=1.0, hits=1.0, auc=1.0)
    m, above, ties = linkpred.link_metrics(np.ones((n, 3)), pos, neg, hits_k=1)
    assert (above == 0).all() and (ties == K).all()
    assert m["mean_rank"] == 1.0 and m["auc"] == 0.5


def test_holdout_removes_exactly_the_held_out_edges():
    g, _ = workload("tiny")
    tr, pos = holdout_edges(g, 60, seed=7)
    arcs = lambda gr: {(u, int(v)) for u in range(gr.n)
                       for v in gr.col[gr.rowptr[u]:gr.rowptr[u + 1]]}
    a0, a1 = arcs(g), arcs(tr)
    gone = {(int(a), int(b)) for a, b in pos} | {(int(b), int(a)) for a, b in pos}
    assert len(gone) == 120 and gone <= a0
    assert a1 == a0 - gone
    for u in range(tr.n):
        assert np.all(np.diff(tr.col[tr.rowptr[u]:tr.rowptr[u + 1]]) > 0)
    neg = corrupt_destinations(pos, g.n, 30, seed=8)
    assert neg.shape == (60, 30) and np.all(neg != pos[:, 1:2])
    assert neg.min() >= 0 and neg.max() < g.n
