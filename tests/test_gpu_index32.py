"""Graphs passed with 32-bit row offsets (lne_graph.index_bits = 32): the
count matrix is bit-exact with the oracle's, and every entry point that takes
a graph returns bit for bit what it returns for the same graph with 64-bit
offsets (the 64-bit path is checked against the oracle by the other tests)."""
import math

import numpy as np
import pytest
import torch

import oracle
from synth import chung_lu, sbm, trial_vectors
from tests import graphs_small as gs
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu


def both(g):
    rp, col = to_dev(g)
    return rp, rp.to(torch.int32), col


@pytest.mark.parametrize("name", ["kite", "sbm"])
def test_counts_index32_bit_exact_with_oracle(lne, ctx, name):
    g = gs.kite() if name == "kite" else sbm([40, 40, 40], 0.2, 0.02, seed=4)
    p = gs.params(T=4, M_per_m=30, C=math.log(g.n), m=g.m, seed=5)
    _, rp32, col = both(g)
    csr, st = lne.sparsify(ctx, rp32, col, p)
    R, C, W = (x.cpu().numpy() for x in csr.to_torch())
    R0, C0, W0, att, acc = oracle.count_csr(g, p)
    np.testing.assert_array_equal(R, R0)
    np.testing.assert_array_equal(C, C0)
    np.testing.assert_array_equal(W.view(np.uint64), W0)
    assert (st["attempted"], st["accepted"]) == (att, acc)


def test_index32_equals_index64(lne, ctx):
    g = chung_lu(3000, 30000, 2.1, seed=3)          # hubs and isolated vertices
    rp, rp32, col = both(g)
    p = dict(T=5, s=[0.2] * 5, M=4 * 5 * g.m, b=1, C=math.log(g.n), d=16, oversample=8, q=1,
             cheb_k=6, theta=0.5, mu=0.2, seed=11, precision="f32")
    print("embed f32", flush=True)
    X64, s64 = lne.embed(ctx, rp, col, p)
    X32, s32 = lne.embed(ctx, rp32, col, p)
    assert s64 == s32
    assert torch.equal(X64, X32)
    print("sparsify_log", flush=True)
    M64, _ = lne.sparsify_log(ctx, rp, col, p)
    M32, _ = lne.sparsify_log(ctx, rp32, col, p)
    for a, b in zip(M64.to_torch(), M32.to_torch()):
        assert torch.equal(a, b)
    print("graph_spmm / propagate", flush=True)
    Z = torch.randn(g.n, 16, dtype=torch.float32, device="cuda")
    assert torch.equal(lne.graph_spmm(ctx, rp, col, Z, 0.7, -1.0),
                       lne.graph_spmm(ctx, rp32, col, Z, 0.7, -1.0))
    assert torch.equal(lne.propagate(ctx, rp, col, p, Z), lne.propagate(ctx, rp32, col, p, Z))
    print("graph_stats", flush=True)
    np.testing.assert_array_equal(lne.graph_stats(ctx, rp, col, seed=2, wedges=500, iters=30),
                                  lne.graph_stats(ctx, rp32, col, seed=2, wedges=500, iters=30))
    print("embed_batch", flush=True)
    trials = trial_vectors(3, seed=1, T=5)
    B64, _ = lne.embed_batch(ctx, rp, col, p, trials)
    B32, _ = lne.embed_batch(ctx, rp32, col, p, trials)
    assert torch.equal(B64, B32)
