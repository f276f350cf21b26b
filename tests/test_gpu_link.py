"""GPU link-prediction ranking (lne_link_rank) against the FP64 oracle, and the
whole evaluation protocol: hold out edges, embed the training graph, rank."""
import numpy as np
import pytest

from oracle import linkpred
from synth import workload, holdout_edges, corrupt_destinations
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu


def _bands(X, pos, neg):
    """Per edge: corrupted edges surely above, surely below and too close to
    call given FP64 rounding of d-term sums taken in any order."""
    sp = linkpred.scores(X, pos[:, 0], pos[:, 1])
    sn = linkpred.scores(X, pos[:, 0][:, None], neg)
    nu = np.linalg.norm(X[pos[:, 0]], axis=1)[:, None]
    scale = nu * (np.linalg.norm(X[neg], axis=2) + np.linalg.norm(X[pos[:, 1]], axis=1)[:, None])
    eps = 1e-12 * scale
    diff = sn - sp[:, None]
    return (diff > eps).sum(1), (diff < -eps).sum(1), (np.abs(diff) <= eps).sum(1)


def _case(seed, n, d, h, K, integer=False):
    rng = np.random.default_rng(seed)
    if integer:
        X = rng.integers(-2, 3, size=(n, d)).astype(np.float64)
    else:
        X = rng.standard_normal((n, d))
    pos = np.stack([rng.integers(0, n, h), rng.integers(0, n, h)], axis=1).astype(np.int32)
    neg = corrupt_destinations(pos, n, K, seed + 1)
    return X, pos, neg


def _dev(X, dtype, ld):
    import torch
    n, d = X.shape
    Xd = torch.zeros((n, ld), dtype=dtype, device="cuda")
    Xd[:, :d] = torch.from_numpy(X).to(dtype)
    return Xd[:, :d]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("d,K", [(32, 300), (130, 77)])
def test_link_rank_matches_oracle(lne, ctx, prec, d, K):
    import torch
    X, pos, neg = _case(3 + d, n=4000, d=d, h=257, K=K)
    dt = torch.float64 if prec == "f64" else torch.float32
    Xd = _dev(X, dt, (d + 3) // 4 * 4)
    Xq = Xd.double().cpu().numpy()                 # the values the GPU sees
    m, above, ties = lne.link_rank(ctx, Xd, torch.from_numpy(pos).cuda(),
                                   torch.from_numpy(neg).cuda(), hits_k=10)
    above = above.cpu().numpy()
    ties = ties.cpu().numpy()
    sure_above, sure_below, amb = _bands(Xq, pos, neg)
    assert np.all(above >= sure_above) and np.all(above + ties <= K - sure_below)
    assert np.all(above <= sure_above + amb)
    ref = linkpred.metrics(above, ties, K, 10)
    for key in ref:
        assert m[key] == pytest.approx(ref[key], rel=1e-12, abs=1e-12)
    if amb.sum() == 0:
        exact, _, _ = linkpred.link_metrics(Xq, pos, neg, 10)
        assert m == pytest.approx(exact, rel=1e-12, abs=1e-12)


def test_link_rank_integer_embedding_exact_with_ties(lne, ctx):
    import torch
    X, pos, neg = _case(11, n=500, d=6, h=200, K=90, integer=True)
    Xd = _dev(X, torch.float32, 8)
    m, above, ties = lne.link_rank(ctx, Xd, torch.from_numpy(pos).cuda(),
                                   torch.from_numpy(neg).cuda(), hits_k=5)
    ref, ra, rt = linkpred.link_metrics(X, pos, neg, 5)
    np.testing.assert_array_equal(above.cpu().numpy(), ra)
    np.testing.assert_array_equal(ties.cpu().numpy(), rt)
    assert rt.sum() > 0
    assert m == pytest.approx(ref, rel=1e-13, abs=1e-13)


def test_link_rank_rejects_out_of_range_ids(lne, ctx):
    import torch
    X, pos, neg = _case(5, n=100, d=8, h=10, K=20)
    neg[3, 7] = 100
    with pytest.raises(lne.LneError):
        lne.link_rank(ctx, _dev(X, torch.float32, 8), torch.from_numpy(pos).cuda(),
                      torch.from_numpy(neg).cuda())
    pos[0, 1] = -1
    with pytest.raises(lne.LneError):
        lne.link_rank(ctx, _dev(X, torch.float32, 8), torch.from_numpy(pos).cuda(),
                      torch.from_numpy(neg).cuda())


def test_link_prediction_protocol_end_to_end(lne, ctx):
    """Held-out edges of a power-law graph rank far above corrupted ones under
    the embedding of the training graph (and not under a random one); the
    library's metrics equal the oracle's on the same embedding."""
    import torch
    g, p = workload("mid")
    train, pos = holdout_edges(g, 400, seed=21)
    neg = corrupt_destinations(pos, g.n, 100, seed=22)
    rp, col = to_dev(train)
    p = dict(p, precision="f32", d=32, T=2, s=[0.5, 0.5], cheb_k=0, M=200 * 2 * train.m)
    X, _ = lne.embed(ctx, rp, col, p)
    pd, nd = torch.from_numpy(pos).cuda(), torch.from_numpy(neg).cuda()
    m, above, ties = lne.link_rank(ctx, X, pd, nd, hits_k=10)
    Xq = X.double().cpu().numpy()
    sure_above, sure_below, amb = _bands(Xq, pos, neg)
    a = above.cpu().numpy()
    assert np.all(a >= sure_above) and np.all(a <= sure_above + amb)
    ref = linkpred.metrics(a, ties.cpu().numpy(), 100, 10)
    assert m == pytest.approx(ref, rel=1e-12, abs=1e-12)
    Xr = torch.randn_like(X)
    mr, _, _ = lne.link_rank(ctx, Xr, pd, nd, hits_k=10)
    print("embedding", m, "random", mr)
    assert m["auc"] > mr["auc"] + 0.15
    assert m["mrr"] > 2 * mr["mrr"]
