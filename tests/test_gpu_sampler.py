"""GPU sparsifier vs the oracle: sample slots, count CSR and trunc_log
structure bit-exact; trunc_log values within a few ulp."""
import math

import numpy as np
import pytest

import oracle
from synth import sbm, workload
from tests import graphs_small as gs
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu


def _slots_parity(lne, ctx, g, p, e0, e1):
    rp, col = to_dev(g)
    out = lne.sample_slots(ctx, rp, col, p, e0, e1)
    S = out["S"]
    ref = oracle.sample_slots(g, p, e0, e1)
    a = out["a"].cpu().numpy().reshape(-1, S)
    b = out["b"].cpu().numpy().reshape(-1, S)
    w = out["w"].cpu().numpy().view(np.uint64).reshape(-1, S)
    r = out["r"].cpu().numpy().reshape(-1, S)
    e = ref["e"] - e0
    j = ref["j"].astype(np.int64)
    np.testing.assert_array_equal(a[e, j], ref["a"])
    np.testing.assert_array_equal(b[e, j], ref["b"])
    np.testing.assert_array_equal(w[e, j], ref["w"])
    np.testing.assert_array_equal(r[e, j], ref["r"])
    # slots beyond n_e are empty
    filled = np.zeros_like(a, dtype=bool)
    filled[e, j] = True
    assert np.all(a[~filled] == -1) and np.all(w[~filled] == 0) and np.all(r[~filled] == 0)
    return len(ref["e"])


@pytest.mark.parametrize("C", [None, "ln", 0.7])
def test_sample_slots_tiny_graphs(lne, ctx, C):
    for g in (gs.kite(), gs.star(6), gs.path(5), gs.complete(6)):
        cval = math.log(g.n) if C == "ln" else C
        p = gs.params(T=5, s=[0.1, 0.3, 0.2, 0.25, 0.15], M_per_m=37, C=cval, m=g.m, seed=5)
        p["M"] += 3           # fractional M/m: Bernoulli extra slot
        _slots_parity(lne, ctx, g, p, 0, g.m)


def test_sample_slots_tiny_workload_ranges(lne, ctx):
    g, p = workload("tiny")
    for e0, e1 in [(0, 50), (4000, 4100), (g.m - 7, g.m)]:
        assert _slots_parity(lne, ctx, g, p, e0, e1) > 0


def _count_parity(lne, ctx, g, p):
    rp, col = to_dev(g)
    csr, st = lne.sparsify(ctx, rp, col, p)
    R, C, W = (x.cpu().numpy() for x in csr.to_torch())
    R0, C0, W0, att, acc = oracle.count_csr(g, p)
    np.testing.assert_array_equal(R, R0)
    np.testing.assert_array_equal(C, C0)
    np.testing.assert_array_equal(W.view(np.uint64), W0)
    assert st["attempted"] == att and st["accepted"] == acc
    return csr


@pytest.mark.parametrize("name", ["kite", "star", "K6", "isolated", "single"])
def test_count_csr_small_graphs(lne, ctx, name):
    g = {"kite": gs.kite(), "star": gs.star(9), "K6": gs.complete(6),
         "isolated": gs.from_edges(12, [(1, 4), (4, 9), (9, 1), (2, 3)]),
         "single": gs.from_edges(3, [(0, 2)])}[name]
    for C in (None, math.log(g.n), 0.4):
        p = gs.params(T=4, s=[0.4, 0.3, 0.2, 0.1], M_per_m=25, C=C, m=g.m, seed=7)
        p["M"] += 1
        _count_parity(lne, ctx, g, p)


def test_count_csr_fewer_samples_than_edges(lne, ctx):
    g = sbm([40, 40], 0.3, 0.05, seed=3)
    p = gs.params(T=3, s=[0.5, 0.25, 0.25], M_per_m=1, C=math.log(g.n), m=g.m, seed=2)
    p["M"] = g.m // 3          # n_e is 0 or 1
    _count_parity(lne, ctx, g, p)


def test_count_csr_tiny_workload(lne, ctx):
    g, p = workload("tiny")
    csr = _count_parity(lne, ctx, g, p)
    assert csr.nnz > 100_000


def test_count_csr_deterministic(lne, ctx):
    g, p = workload("tiny")
    rp, col = to_dev(g)
    a, _ = lne.sparsify(ctx, rp, col, p)
    b, _ = lne.sparsify(ctx, rp, col, p)
    for x, y in zip(a.to_torch(), b.to_torch()):
        assert bool((x == y).all())


def test_trunc_log_parity(lne, ctx):
    g, p = workload("tiny")
    rp, col = to_dev(g)
    counts, _ = lne.sparsify(ctx, rp, col, p)
    R0, C0, W0, _, _ = oracle.count_csr(g, p)
    keep, val = oracle.trunc_log(g, p, R0, C0, W0)
    rk, ck, vk = oracle.compact(R0, C0, keep, val)
    for prec, dt, tol_ulp in (("f64", np.float64, 2), ("f32", np.float32, 1)):
        M = lne.trunc_log(ctx, rp, col, dict(p, precision=prec), counts)
        R, C, V = (x.cpu().numpy() for x in M.to_torch())
        np.testing.assert_array_equal(R, rk)
        np.testing.assert_array_equal(C, ck)
        ref = vk.astype(dt)
        ulp = np.spacing(np.abs(ref).astype(dt))
        assert np.all(np.abs(V.astype(np.float64) - ref.astype(np.float64)) <= tol_ulp * ulp + 1e-300)


def test_trunc_log_strict_boundary(lne, ctx):
    k44 = gs.from_edges(8, [(i, j) for i in range(4) for j in range(4, 8)])
    p = gs.params(T=1, s=[1.0], M_per_m=5, C=None, m=k44.m, b=2)
    rp, col = to_dev(k44)
    counts, _ = lne.sparsify(ctx, rp, col, p)
    M = lne.trunc_log(ctx, rp, col, p, counts)
    assert counts.nnz == 32 and M.nnz == 0


def test_row_range_passes_match_single_pass(lne, ctx, monkeypatch):
    """A pair-buffer budget far below the need splits the rows into ranges
    (each range re-walks every sample); the result is identical."""
    g, p = workload("tiny")
    rp, col = to_dev(g)
    ref, st_ref = lne.sparsify(ctx, rp, col, p)
    R0, C0, W0 = (x.cpu().numpy() for x in ref.to_torch())
    Xref, _ = lne.embed(ctx, rp, col, p)
    monkeypatch.setenv("LNE_HBM_BUDGET_GB", "0.05")
    csr, st = lne.sparsify(ctx, rp, col, p)
    R, C, W = (x.cpu().numpy() for x in csr.to_torch())
    np.testing.assert_array_equal(R, R0)
    np.testing.assert_array_equal(C, C0)
    np.testing.assert_array_equal(W, W0)
    assert st == st_ref
    X, _ = lne.embed(ctx, rp, col, p)
    assert bool((X == Xref).all())


def _compact(R, C, V):
    """Drop explicit zeros from a CSR (numpy)."""
    keep = V != 0
    rows = np.repeat(np.arange(len(R) - 1), np.diff(R))
    R2 = np.zeros_like(R)
    np.add.at(R2, rows[keep] + 1, 1)
    return np.cumsum(R2), C[keep], V[keep]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("budget", [None, "0.05"])
def test_embedding_matrix_equals_trunc_log_of_counts(lne, ctx, monkeypatch, prec, budget):
    """The matrix the embedding factorises (Eq. (1) fused into the aggregation,
    degrees carried in the sort keys) equals lne_trunc_log of the count matrix
    entry for entry, explicit zeros aside; in one block and in row ranges."""
    g, p = workload("tiny")
    p = dict(p, precision=prec)
    rp, col = to_dev(g)
    if budget:
        monkeypatch.setenv("LNE_HBM_BUDGET_GB", budget)
    counts, st0 = lne.sparsify(ctx, rp, col, p)
    M0 = lne.trunc_log(ctx, rp, col, p, counts)
    R0, C0, V0 = (x.cpu().numpy() for x in M0.to_torch())
    M1, st1 = lne.sparsify_log(ctx, rp, col, p)
    R1, C1, V1 = _compact(*(x.cpu().numpy() for x in M1.to_torch()))
    assert st1["nnz_log"] == M0.nnz and st1["accepted"] == st0["accepted"]
    np.testing.assert_array_equal(R1, R0)
    np.testing.assert_array_equal(C1, C0)
    np.testing.assert_array_equal(V1, V0)


def test_embedding_matrix_weighted_and_hub(lne, ctx):
    """Weighted degrees in the keys' tags, and a hub whose degree (70,000)
    does not fit a tag: looked up instead."""
    from tests.test_gpu_weighted import _dev_w
    g, p = workload("tiny")
    gw = gs.with_weights(g, 5)
    rp, col = to_dev(gw)
    counts, _ = lne.sparsify(ctx, rp, col, p, weight=_dev_w(gw))
    M0 = lne.trunc_log(ctx, rp, col, p, counts, weight=_dev_w(gw))
    M1, _ = lne.sparsify_log(ctx, rp, col, p, weight=_dev_w(gw))
    for a, b in zip((x.cpu().numpy() for x in M0.to_torch()),
                    _compact(*(x.cpu().numpy() for x in M1.to_torch()))):
        np.testing.assert_array_equal(a, b)
    hub = gs.star(70_001)
    ph = gs.params(T=2, s=[0.5, 0.5], M_per_m=4, C=None, m=hub.m, seed=2)
    rp, col = to_dev(hub)
    counts, _ = lne.sparsify(ctx, rp, col, ph)
    M0 = lne.trunc_log(ctx, rp, col, ph, counts)
    M1, _ = lne.sparsify_log(ctx, rp, col, ph)
    assert M0.nnz > 0
    for a, b in zip((x.cpu().numpy() for x in M0.to_torch()),
                    _compact(*(x.cpu().numpy() for x in M1.to_torch()))):
        np.testing.assert_array_equal(a, b)
