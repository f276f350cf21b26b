"""Batched trials sharing one sampling pass: the channel sparsifier is
bit-exact with the oracle, each trial's matrix matches the oracle's mixing of
the channels, and the batched pipeline equals the single-trial pipeline run
on the same trial matrices."""
import math

import numpy as np
import pytest

import oracle
from synth import sbm, trial_vectors, workload
from tests import graphs_small as gs
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu


def procrustes_err(X, Xref):
    U, _, Vt = np.linalg.svd(X.T @ Xref)
    return float(np.linalg.norm(X @ (U @ Vt) - Xref) / np.linalg.norm(Xref))


@pytest.mark.parametrize("C", [None, "ln"])
def test_channel_counts_bit_exact(lne, ctx, C):
    for g in (gs.kite(), sbm([40, 40, 40], 0.2, 0.02, seed=4)):
        p = gs.params(T=6, M_per_m=30, C=(math.log(g.n) if C == "ln" else None), m=g.m, seed=5)
        p["M"] += 7
        rp, col = to_dev(g)
        csr, st = lne.sparsify_channels(ctx, rp, col, p)
        R, Cx, W = (x.cpu().numpy() for x in csr.to_torch())
        R0, C0, W0, att, acc = oracle.count_csr(g, p, channels=True)
        np.testing.assert_array_equal(R, R0)
        np.testing.assert_array_equal(Cx, C0)
        np.testing.assert_array_equal(W.view(np.uint64), W0)
        assert (st["attempted"], st["accepted"]) == (att, acc)


def test_trial_matrix_matches_oracle_mixing(lne, ctx):
    g, p = workload("tiny")
    p = dict(p, M=20 * p["T"] * g.m, precision="f32")
    rp, col = to_dev(g)
    ch, _ = lne.sparsify_channels(ctx, rp, col, p)
    R0, C0, W0, _, _ = oracle.count_csr(g, p, channels=True)
    for tr in trial_vectors(3, seed=2):
        M = lne.trial_matrix(ctx, rp, col, p, ch, tr)
        R, C, V = (x.cpu().numpy() for x in M.to_torch())
        ref = oracle.trial_matrix(g, p, R0, C0, W0, tr["s"])
        np.testing.assert_array_equal(R, ref.indptr)
        np.testing.assert_array_equal(C, ref.indices)
        np.testing.assert_array_equal(V > 0, ref.data > 0)
        np.testing.assert_allclose(V, ref.data.astype(np.float32), rtol=2e-6, atol=1e-6)


def test_batched_pipeline_equals_single_trial_runs(lne, ctx):
    g = sbm([100] * 8, 0.12, 0.01, seed=3)
    p = dict(T=10, s=np.full(10, 0.1), M=30 * 10 * g.m, b=1, C=math.log(g.n), d=16,
             oversample=8, q=2, cheb_k=5, theta=0.5, mu=0.2, seed=1, precision="f32")
    rp, col = to_dev(g)
    trials = trial_vectors(5, seed=7)
    trials[1]["k"] = 0                      # propagation off for one trial
    Xb, st = lne.embed_batch(ctx, rp, col, p, trials)
    ch, _ = lne.sparsify_channels(ctx, rp, col, p)
    for t, tr in enumerate(trials):
        M = lne.trial_matrix(ctx, rp, col, p, ch, tr)
        pt = dict(p, s=tr["s"], cheb_k=tr["k"], theta=tr["theta"], mu=tr["mu"])
        U, S, V, X0 = lne.rsvd(ctx, M, pt)
        X = lne.propagate(ctx, rp, col, pt, X0).cpu().numpy()
        err = procrustes_err(Xb[t].cpu().numpy(), X)
        assert err < 2e-3, (t, err)
