"""Weighted graphs on the GPU against the oracle: every sample slot (walk by
weight, path factor, degree sampling with A_uv) and the count matrix bit for
bit, Eq. (1) with weighted degrees and vol, the weighted propagation and the
whole embedding; unit weights reproduce the unweighted path exactly."""
import math

import numpy as np
import pytest

import oracle
from synth import workload
from tests import graphs_small as gs
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu


def _dev_w(g):
    import torch
    return torch.from_numpy(g.weight.astype(np.int32)).cuda()


def procrustes_err(X, Xref):
    U, _, Vt = np.linalg.svd(X.T @ Xref)
    return float(np.linalg.norm(X @ (U @ Vt) - Xref) / np.linalg.norm(Xref))


@pytest.fixture(scope="module")
def wtiny():
    g, p = workload("tiny")
    return gs.with_weights(g, 17), p


@pytest.mark.parametrize("C", [None, 0.6])
def test_weighted_slots_bit_exact(lne, ctx, C):
    g = gs.with_weights(gs.kite(), 3)
    p = gs.params(T=4, s=[0.1, 0.4, 0.3, 0.2], M_per_m=40, C=C, m=g.m, seed=5)
    p["M"] += 3                      # fractional M/m: Bernoulli extra slot
    rp, col = to_dev(g)
    out = lne.sample_slots(ctx, rp, col, p, 0, g.m, weight=_dev_w(g))
    S = out["S"]
    ref = oracle.sample_slots(g, p)
    a = out["a"].cpu().numpy().reshape(-1, S)
    b = out["b"].cpu().numpy().reshape(-1, S)
    w = out["w"].cpu().numpy().view(np.uint64).reshape(-1, S)
    r = out["r"].cpu().numpy().reshape(-1, S)
    e, j = ref["e"], ref["j"].astype(np.int64)
    np.testing.assert_array_equal(a[e, j], ref["a"])
    np.testing.assert_array_equal(b[e, j], ref["b"])
    np.testing.assert_array_equal(w[e, j], ref["w"])
    np.testing.assert_array_equal(r[e, j], ref["r"])
    acc = ref["acc"].astype(bool)
    assert len(np.unique(ref["w"][acc])) > 3        # path-dependent weights


def _skewed(g, seed):
    """g with symmetric weights 2^j, j uniform in 0..20: slices of one row
    differ by up to 2^20, so a guide bucket can hold many slices or a slice
    many buckets."""
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    key = np.minimum(rows, g.col).astype(np.int64) * g.n + np.maximum(rows, g.col)
    _, inv = np.unique(key, return_inverse=True)
    w = (1 << rng.integers(0, 21, size=inv.max() + 1)).astype(np.uint32)[inv]
    return type(g)(g.n, g.rowptr, g.col, g.labels, g.name + "-skew", w)


@pytest.mark.parametrize("graph", ["star", "tiny"])
def test_weighted_slots_skewed_weights_bit_exact(lne, ctx, graph):
    """Walk steps by weight on rows whose slices span six orders of
    magnitude (a 300-leaf star's hub, a planted-block graph)."""
    g = gs.star(300) if graph == "star" else workload("tiny")[0]
    g = _skewed(g, 9)
    p = gs.params(T=6, s=[0.1, 0.2, 0.2, 0.2, 0.2, 0.1], M_per_m=20, C=None, m=g.m, seed=3)
    rp, col = to_dev(g)
    out = lne.sample_slots(ctx, rp, col, p, 0, g.m, weight=_dev_w(g))
    S = out["S"]
    ref = oracle.sample_slots(g, p)
    e, j = ref["e"], ref["j"].astype(np.int64)
    for key in ("a", "b", "r"):
        np.testing.assert_array_equal(out[key].cpu().numpy().reshape(-1, S)[e, j], ref[key])
    w = out["w"].cpu().numpy().view(np.uint64).reshape(-1, S)
    np.testing.assert_array_equal(w[e, j], ref["w"])


def test_weighted_counts_and_trunc_log(lne, ctx, wtiny):
    g, p = wtiny
    rp, col = to_dev(g)
    wd = _dev_w(g)
    counts, st = lne.sparsify(ctx, rp, col, p, weight=wd)
    R, C, W = (x.cpu().numpy() for x in counts.to_torch())
    Ro, Co, Wo, att, acc = oracle.count_csr(g, p)
    np.testing.assert_array_equal(R, Ro)
    np.testing.assert_array_equal(C, Co)
    np.testing.assert_array_equal(W.view(np.uint64), Wo)
    assert st["accepted"] == acc and st["attempted"] == att
    M = lne.trunc_log(ctx, rp, col, p, counts, weight=wd)
    keep, val = oracle.trunc_log(g, p, Ro, Co, Wo)
    R2, C2, V2 = (x.cpu().numpy() for x in M.to_torch())
    rows = np.repeat(np.arange(g.n), np.diff(Ro))
    ref = np.zeros((g.n, g.n))
    ref[rows[keep], Co[keep]] = val[keep]
    assert M.nnz == int(keep.sum())
    got = np.zeros((g.n, g.n))
    got[np.repeat(np.arange(g.n), np.diff(R2)), C2] = V2
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-14)


def test_weighted_propagation_matches_oracle(lne, ctx, wtiny):
    import torch
    g, p = wtiny
    rp, col = to_dev(g)
    X0 = np.random.default_rng(4).standard_normal((g.n, 24))
    pp = dict(p, d=24, cheb_k=6, theta=0.6, mu=0.15, flags=lne.FLAG_NO_FINAL_EIGSVD)
    for prec, tol in (("f64", 1e-12), ("f32", 1e-5)):
        tdt = torch.float64 if prec == "f64" else torch.float32
        X0d = torch.from_numpy(X0).to(tdt).cuda()
        X = lne.propagate(ctx, rp, col, dict(pp, precision=prec), X0d,
                          weight=_dev_w(g)).double().cpu().numpy()
        ref = oracle.propagate(g, X0d.double().cpu().numpy(), 6, 0.6, 0.15)
        assert np.max(np.abs(X - ref)) <= tol * np.max(np.abs(X0)) * 13


def test_weighted_embedding_matches_oracle(lne, ctx, wtiny):
    g, p = wtiny
    rp, col = to_dev(g)
    X, st = lne.embed(ctx, rp, col, p, weight=_dev_w(g))
    ref = oracle.embed(g, p, return_stages=True)
    assert st["nnz_log"] == ref["M"].nnz
    assert procrustes_err(X.cpu().numpy(), ref["X"]) < 1e-8


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_unit_weights_reproduce_unweighted_path(lne, ctx, prec):
    import torch
    g, p = workload("tiny")
    p = dict(p, precision=prec)
    rp, col = to_dev(g)
    ones = torch.ones(g.n_arcs, dtype=torch.int32, device="cuda")
    X0, s0 = lne.embed(ctx, rp, col, p)
    X1, s1 = lne.embed(ctx, rp, col, p, weight=ones)
    assert s0 == s1
    assert torch.equal(X0, X1)


def test_weight_errors(lne, ctx):
    import torch
    g, p = workload("tiny")
    rp, col = to_dev(g)
    w = torch.ones(g.n_arcs, dtype=torch.int32, device="cuda")
    w[5] = 0
    with pytest.raises(lne.LneError):
        lne.embed(ctx, rp, col, p, weight=w)
    w[5] = 1
    big = torch.full((g.n_arcs,), 2 ** 31 - 1, dtype=torch.int32, device="cuda")
    with pytest.raises(lne.LneError):          # vol beyond 2^32
        lne.sparsify(ctx, rp, col, p, weight=big)
