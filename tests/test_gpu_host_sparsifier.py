"""The sparsifier kept in pinned host memory (LNE_FLAG_HOST_SPARSIFIER, the
path for graphs whose sparsified matrix exceeds HBM): every product of the
randomized SVD streams the row chunks over PCIe.  With the dense Gaussian
test matrix the rows of each product are computed by the same kernel on the
same entries in the same order, so the embedding is bit-identical to the
in-HBM path, whatever the chunking and row-range split; with the sparse-sign
test matrix (LDS atomics, order free) it matches the oracle."""
import numpy as np
import pytest

import oracle
from synth import workload, pair_weights
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu


def _same(lne, ctx, rp, col, p, weight=None):
    X0, st0 = lne.embed(ctx, rp, col, p, weight=weight)
    X1, st1 = lne.embed(ctx, rp, col, dict(p, flags=p.get("flags", 0) | lne.FLAG_HOST_SPARSIFIER),
                        weight=weight)
    assert st1 == st0
    assert X1.dtype == X0.dtype and bool((X1 == X0).all())
    return X1


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("chunk", ["100", "5000", "1000000000"])   # 100: most rows alone
def test_host_sparsifier_bit_identical(lne, ctx, monkeypatch, prec, chunk):
    print("host sparsifier: tiny", prec, "chunk", chunk, flush=True)
    g, p = workload("tiny")
    rp, col = to_dev(g)
    monkeypatch.setenv("LNE_HOST_CHUNK_NNZ", chunk)
    _same(lne, ctx, rp, col, dict(p, precision=prec))


def test_host_sparsifier_with_row_ranges(lne, ctx, monkeypatch):
    """Several sparsifier row blocks (pair budget far below the need), each
    cut into several chunks."""
    g, p = workload("tiny")
    rp, col = to_dev(g)
    monkeypatch.setenv("LNE_HBM_BUDGET_GB", "0.05")
    monkeypatch.setenv("LNE_HOST_CHUNK_NNZ", "3000")
    _same(lne, ctx, rp, col, p)


def test_host_sparsifier_power_law_f32(lne, ctx, monkeypatch):
    g, p = workload("mid")
    rp, col = to_dev(g)
    monkeypatch.setenv("LNE_HOST_CHUNK_NNZ", str(1 << 20))
    _same(lne, ctx, rp, col, dict(p, M=20 * 2 * g.m))


def test_host_sparsifier_vanilla_rsvd_and_weights(lne, ctx, monkeypatch):
    import torch
    g, p = workload("tiny")
    rp, col = to_dev(g)
    monkeypatch.setenv("LNE_HOST_CHUNK_NNZ", "7000")
    _same(lne, ctx, rp, col, dict(p, q=2, flags=lne.FLAG_VANILLA_RSVD))
    w = torch.from_numpy(pair_weights(g, 5, seed=3).astype(np.int32)).cuda()
    _same(lne, ctx, rp, col, p, weight=w)


def test_host_sparsifier_sparse_omega_matches_oracle(lne, ctx, monkeypatch):
    from tests.test_gpu_linalg import procrustes_err
    g, p = workload("tiny")
    rp, col = to_dev(g)
    monkeypatch.setenv("LNE_HOST_CHUNK_NNZ", "4000")
    pp = dict(p, flags=lne.FLAG_SPARSE_OMEGA | lne.FLAG_HOST_SPARSIFIER)
    X, _ = lne.embed(ctx, rp, col, pp)
    ref = oracle.embed(g, dict(p, flags=lne.FLAG_SPARSE_OMEGA))
    assert procrustes_err(X.cpu().numpy(), ref) < 1e-8
