"""Batched trials sharing one sampling pass: the channel sparsifier is
bit-exact with the oracle, each trial's matrix matches the oracle's mixing of
the channels, the batched SpMM (values generated on the fly) matches the
oracle's trial matrix times the operand, and the batched pipeline -- eager or
replayed from a captured HIP graph -- equals the single-trial pipeline run on
the same trial matrices."""
import json
import math

import numpy as np
import pytest

import oracle
from synth import sbm, trial_vectors, workload
from tests import bars
from tests import graphs_small as gs
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu


def procrustes_err(X, Xref):
    U, _, Vt = np.linalg.svd(X.T @ Xref)
    return float(np.linalg.norm(X @ (U @ Vt) - Xref) / np.linalg.norm(Xref))


@pytest.mark.parametrize("C,pi", [(None, None), ("ln", None), ("ln", [3, 1, 0.5, 2, 0.2, 1])])
def test_channel_counts_bit_exact(lne, ctx, C, pi):
    for g in (gs.kite(), sbm([40, 40, 40], 0.2, 0.02, seed=4)):
        p = gs.params(T=6, s=pi, M_per_m=30, C=(math.log(g.n) if C == "ln" else None), m=g.m,
                      seed=5)
        p["M"] += 7
        rp, col = to_dev(g)
        csr, st = lne.sparsify_channels(ctx, rp, col, p)
        R, Cx, W = (x.cpu().numpy() for x in csr.to_torch())
        R0, C0, W0, att, acc = oracle.count_csr(g, p, channels=True)
        np.testing.assert_array_equal(R, R0)
        np.testing.assert_array_equal(Cx, C0)
        np.testing.assert_array_equal(W.view(np.uint64), W0)
        assert (st["attempted"], st["accepted"]) == (att, acc)


@pytest.mark.parametrize("skew", [False, True])
def test_trial_matrix_matches_oracle_mixing(lne, ctx, skew):
    g, p = workload("tiny")
    p = dict(p, M=20 * p["T"] * g.m, precision="f32")
    if skew:
        p["s"] = np.linspace(1.0, 3.0, p["T"])
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


def _spmm_bar(M, X):
    """FP32 accumulation bound: |M| |X| per entry times a few ulps per term."""
    absmx = abs(M) @ np.abs(X)
    nnz_row = np.diff(M.indptr).max()
    return 4 * max(nnz_row, 1) * 2.0 ** -24 * absmx + 1e-30


def test_batch_spmm_matches_oracle(lne, ctx):
    """Values generated inside the SpMM equal the oracle's trial matrices:
    per-trial and shared operands, widths that leave lanes idle and fill the
    wave, rows longer than one 64-entry chunk (channel runs straddle chunks)."""
    import torch
    g = sbm([150] * 4, 0.3, 0.02, seed=8)
    p = gs.params(T=8, M_per_m=60, C=math.log(g.n), m=g.m, seed=3, d=16, oversample=8,
                  precision="f32")
    rp, col = to_dev(g)
    R0, C0, W0, _, _ = oracle.count_csr(g, p, channels=True)
    assert np.diff(R0).max() > 200
    trials = trial_vectors(3, seed=4, T=8)
    trials[2]["s"] = np.array([0, 0, 1.0, 0, 0, 0, 0, 0])     # one length only
    B = lne.Batch(ctx, rp, col, p, max_trials=3)
    Ms = [oracle.trial_matrix(g, p, R0, C0, W0, tr["s"]) for tr in trials]
    rng = np.random.default_rng(0)
    for k in (4, 36, 144, 256):
        X = rng.standard_normal((3, g.n, k)).astype(np.float32)
        Y = B.spmm(trials, torch.from_numpy(X).cuda()).cpu().numpy()
        for t in range(3):
            ref = Ms[t] @ X[t].astype(np.float64)
            bar = _spmm_bar(Ms[t], X[t].astype(np.float64))
            assert np.all(np.abs(Y[t] - ref) <= bar), (k, t, np.max(np.abs(Y[t] - ref) / bar))
    Xs = rng.standard_normal((g.n, 32)).astype(np.float32)
    Y = B.spmm(trials, torch.from_numpy(Xs).cuda()).cpu().numpy()
    for t in range(3):
        ref = Ms[t] @ Xs.astype(np.float64)
        assert np.all(np.abs(Y[t] - ref) <= _spmm_bar(Ms[t], Xs.astype(np.float64)))
    # a channel pass drawn from another length distribution: same contract
    pi = np.array([0.05, 0.1, 0.3, 0.2, 0.1, 0.1, 0.1, 0.05])
    B.resample(pi)
    R1, C1, W1, _, _ = oracle.count_csr(g, dict(p, s=pi), channels=True)
    assert B.info()["channel_nnz"] == len(C1)
    X = rng.standard_normal((3, g.n, 36)).astype(np.float32)
    Y = B.spmm(trials, torch.from_numpy(X).cuda()).cpu().numpy()
    for t in range(3):
        M = oracle.trial_matrix(g, dict(p, s=pi), R1, C1, W1, trials[t]["s"])
        ref = M @ X[t].astype(np.float64)
        assert np.all(np.abs(Y[t] - ref) <= _spmm_bar(M, X[t].astype(np.float64)))
    B.close()


def _single_trial_reference(lne, ctx, rp, col, p, ch, tr):
    M = lne.trial_matrix(ctx, rp, col, p, ch, tr)
    pt = dict(p, s=tr["s"], cheb_k=tr["k"], theta=tr["theta"], mu=tr["mu"])
    U, S, V, X0 = lne.rsvd(ctx, M, pt)
    return lne.propagate(ctx, rp, col, pt, X0).cpu().numpy()


def test_batched_pipeline_equals_single_trial_runs(lne, ctx):
    g = sbm([100] * 8, 0.12, 0.01, seed=3)
    p = dict(T=10, s=np.full(10, 0.1), M=30 * 10 * g.m, b=1, C=math.log(g.n), d=16,
             oversample=8, q=2, cheb_k=5, theta=0.5, mu=0.2, seed=1, precision="f32")
    rp, col = to_dev(g)
    trials = trial_vectors(5, seed=7)
    trials[1]["k"] = 0                      # propagation off for one trial
    trials[3]["theta"] = 0.0                # and off through theta for another
    Xb, st = lne.embed_batch(ctx, rp, col, p, trials)
    ch, _ = lne.sparsify_channels(ctx, rp, col, p)
    for t, tr in enumerate(trials):
        X = _single_trial_reference(lne, ctx, rp, col, p, ch, tr)
        err = procrustes_err(Xb[t].cpu().numpy(), X)
        assert err < 2e-3, (t, err)


def test_batched_pipeline_matches_oracle(lne, ctx):
    """The batched path end to end (channel pass, values generated inside the
    batched SpMM, batched Gram / Cholesky / eigen-solve / projections,
    batched propagation, final eigSVD) against the FP64 oracle run trial by
    trial: its trial_matrix of the same channel pass, the fast randomized SVD
    with the same Omega, the Chebyshev propagation and the final eigSVD
    (sections 4.2-4.4).  Five trials, one with k = 0 and one with theta = 0
    (propagation off).  d = 8 is the number of planted blocks, where the
    spectrum has its gap; the bar is derived per trial from the oracle's
    quantities (tests/bars.py)."""
    g = sbm([100] * 8, 0.12, 0.01, seed=3)
    d, ov = 8, 8
    p = dict(T=10, s=np.full(10, 0.1), M=30 * 10 * g.m, b=1, C=math.log(g.n), d=d,
             oversample=ov, q=2, cheb_k=5, theta=0.5, mu=0.2, seed=1, precision="f32")
    rp, col = to_dev(g)
    trials = trial_vectors(5, seed=7)
    trials[1]["k"] = 0
    trials[3]["theta"] = 0.0
    Xb, st = lne.embed_batch(ctx, rp, col, p, trials)
    Xb = Xb.double().cpu().numpy()
    R0, C0, W0, _, _ = oracle.count_csr(g, p, channels=True)
    kp = d + ov
    omega = oracle.gaussian_omega(g.n, kp, p["seed"])
    for t, tr in enumerate(trials):
        Mt = oracle.trial_matrix(g, p, R0, C0, W0, tr["s"])
        U, S, V = oracle.fast_rsvd(Mt, kp, 0, p["q"], omega)
        X0 = oracle.embedding(U[:, :d], S[:d])
        on = tr["k"] > 0 and tr["theta"] >= 1e-12
        Xsp = oracle.propagate(g, X0, tr["k"], tr["theta"], tr["mu"]) if on else None
        X = oracle.final_embedding(Xsp) if on else X0
        bar = bars.embedding_bar(g, X0, Xsp, S, d, kp, tr)
        err = procrustes_err(Xb[t], X)
        print(f"trial {t}: k={tr['k']} theta={tr['theta']:.2f} err {err:.3e} bar {bar:.3e}",
              flush=True)
        assert bar < 0.5
        assert err <= bar, (t, err, bar)


def test_graph_replays_equal_eager_runs(lne, ctx):
    """A captured launch sequence replayed several times, with other eager
    work and host synchronisations in between, gives every replay the eager
    result of the same trials; a batch of other trials (and of another size
    and largest order) triggers a new capture and matches its eager run."""
    import torch
    g = sbm([80] * 6, 0.15, 0.01, seed=11)
    p = dict(T=10, s=np.full(10, 0.1), M=20 * 10 * g.m, b=1, C=math.log(g.n), d=16,
             oversample=8, q=1, cheb_k=5, theta=0.5, mu=0.2, seed=2, precision="f32")
    rp, col = to_dev(g)
    B = lne.Batch(ctx, rp, col, p, max_trials=6)
    set_a = trial_vectors(6, seed=21)
    set_b = trial_vectors(4, seed=22)
    set_b[0]["k"] = 0
    first, _ = B.run(set_a)                       # sizes the scratch arena
    eager_a, _ = B.run(set_a)
    eager_b, _ = B.run(set_b)
    np.testing.assert_array_equal(first.cpu().numpy(), eager_a.cpu().numpy())
    for rep in range(3):
        Xa, _ = B.run(set_a, graph=True)
        junk = torch.randn(1 << 20, device="cuda").sum()      # other eager work
        torch.cuda.synchronize()
        np.testing.assert_allclose(Xa.cpu().numpy(), eager_a.cpu().numpy(), rtol=1e-6, atol=1e-7)
        del junk
    for rep in range(2):
        Xb, _ = B.run(set_b, graph=True)
        torch.cuda.synchronize()
        np.testing.assert_allclose(Xb.cpu().numpy(), eager_b.cpu().numpy(), rtol=1e-6, atol=1e-7)
    assert B.info()["graph_captures"] == 2
    # a new channel pass drops the captured graph; the replay after it
    # matches the eager run on the new channels
    B.resample(np.linspace(2.0, 1.0, 10))
    eager_c, _ = B.run(set_a)
    Xc, _ = B.run(set_a, graph=True)
    np.testing.assert_allclose(Xc.cpu().numpy(), eager_c.cpu().numpy(), rtol=1e-6, atol=1e-7)
    assert B.info()["graph_captures"] == 3
    ch, _ = lne.sparsify_channels(ctx, rp, col, p)
    for t in (0, 3):
        X = _single_trial_reference(lne, ctx, rp, col, p, ch, set_a[t])
        assert procrustes_err(eager_a[t].cpu().numpy(), X) < 2e-3
    B.close()


def test_all_trials_off_is_the_rsvd_embedding(lne, ctx):
    g = sbm([60] * 5, 0.2, 0.01, seed=5)
    p = dict(T=10, s=np.full(10, 0.1), M=20 * 10 * g.m, b=1, C=math.log(g.n), d=8,
             oversample=8, q=1, cheb_k=5, theta=0.5, mu=0.2, seed=4, precision="f32")
    rp, col = to_dev(g)
    trials = trial_vectors(3, seed=9)
    for tr in trials:
        tr["k"] = 0
    Xb, _ = lne.embed_batch(ctx, rp, col, p, trials)
    ch, _ = lne.sparsify_channels(ctx, rp, col, p)
    for t, tr in enumerate(trials):
        M = lne.trial_matrix(ctx, rp, col, p, ch, tr)
        _, _, _, X0 = lne.rsvd(ctx, M, dict(p, s=tr["s"]))
        assert procrustes_err(Xb[t].cpu().numpy(), X0.cpu().numpy()) < 2e-3


def test_trial_outside_the_channel_support_is_rejected(lne, ctx):
    g = sbm([50] * 4, 0.2, 0.02, seed=7)
    p = dict(T=4, s=np.array([1.0, 1.0, 0.0, 1.0]), M=10 * 4 * g.m, b=1, C=math.log(g.n), d=8,
             oversample=8, q=1, cheb_k=3, theta=0.5, mu=0.2, seed=4, precision="f32")
    rp, col = to_dev(g)
    B = lne.Batch(ctx, rp, col, p, max_trials=2)
    ok = {"s": np.array([0.5, 0.5, 0.0, 0.0]), "k": 2, "theta": 0.5, "mu": 0.1}
    bad = {"s": np.array([0.5, 0.0, 0.5, 0.0]), "k": 2, "theta": 0.5, "mu": 0.1}
    B.run([ok])
    with pytest.raises(lne.LneError):
        B.run([ok, bad])
    B.close()


def test_tuner_cache_round_trip(lne, ctx, tmp_path, monkeypatch):
    path = tmp_path / "tune.jsonl"
    monkeypatch.setenv("LNE_TUNE_CACHE", str(path))
    g = sbm([60] * 4, 0.2, 0.02, seed=6)
    p = dict(T=6, s=np.full(6, 1 / 6), M=10 * 6 * g.m, b=1, C=math.log(g.n), d=8,
             oversample=8, q=1, cheb_k=3, theta=0.5, mu=0.2, seed=4, precision="f32")
    rp, col = to_dev(g)
    B1 = lne.Batch(ctx, rp, col, p, max_trials=2)
    i1 = B1.info()
    B1.close()
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert {x["op"] for x in lines} == {"spmm_chan", "graph_spmm_batch"}
    sp = [x for x in lines if x["op"] == "spmm_chan"][0]
    assert sp["variant"] == i1["spmm_variant"] and len(sp["ms"]) == 6
    assert sp["nnz_class"] == math.floor(4 * math.log2(i1["channel_nnz"]))
    B2 = lne.Batch(ctx, rp, col, p, max_trials=2)
    assert B2.info()["spmm_variant"] == i1["spmm_variant"]
    assert len(path.read_text().splitlines()) == 2          # read, not re-tuned
    B2.close()
