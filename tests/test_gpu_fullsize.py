"""Parity at the benchmark's full size: the Chung-Lu graph with 10^7 vertices
and 2*10^8 edges, T = 5, s = (0.3, 0.7, 0, 0, 0), M = 4 T m, C = ln n.  The
oracle cannot walk all 4*10^9 samples, but with walk lengths r <= 2 the rows
of a vertex window only receive samples of edges incident to the window's
closed neighbourhood, which it can: on sampled windows the count rows are
bit-exact (through the row-window entry point and through the whole-matrix
sparsifier), and so are the first rSVD product rows Y = M Omega within the
FP32 accumulation bound."""
import math

import numpy as np
import pytest

import oracle
from synth import workload
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu

WINDOWS = [(123_456, 123_460), (5_000_000, 5_000_004), (9_999_990, 10_000_000)]


@pytest.fixture(scope="module")
def large(lne, ctx):
    g, p = workload("large")
    assert np.all(np.asarray(p["s"])[2:] == 0)        # walk lengths 1 and 2 only
    rp, col = to_dev(g)
    refs = {}
    for lo, hi in WINDOWS:
        nb = set(range(lo, hi))
        for a in range(lo, hi):
            nb.update(g.col[g.rowptr[a]:g.rowptr[a + 1]].tolist())
        arcs = np.concatenate([np.arange(g.rowptr[b], g.rowptr[b + 1]) for b in sorted(nb)])
        print(f"window [{lo}, {hi}): {len(nb)} vertices, {len(arcs)} arcs", flush=True)
        sel = oracle.edge_ids_of(g, arcs)
        refs[(lo, hi)] = oracle.count_csr_edges(g, p, lo, hi, sel)
    return g, p, rp, col, refs


def test_count_rows_bit_exact_at_full_size(lne, ctx, large):
    g, p, rp, col, refs = large
    for (lo, hi), (R0, C0, W0) in refs.items():
        csr, st = lne.sparsify_rows(ctx, rp, col, p, lo, hi)
        R, C, W = (x.cpu().numpy() for x in csr.to_torch())
        csr.free()
        np.testing.assert_array_equal(R, R0)
        np.testing.assert_array_equal(C, C0)
        np.testing.assert_array_equal(W.view(np.uint64), W0)
        assert st["attempted"] == p["M"] and st["nnz_counts"] == len(C0)


def test_first_rsvd_product_rows_at_full_size(lne, ctx, large):
    """Whole-matrix sparsifier -> Eq. (1) -> Omega -> Y = M Omega on the
    device, as the embedding runs it; the window rows of the count matrix are
    bit-exact and the rows of Y match the oracle's M rows times its Omega."""
    import torch
    g, p, rp, col, refs = large
    counts, _ = lne.sparsify(ctx, rp, col, p)
    Rd, Cd, Wd = counts.to_torch()
    M = lne.trunc_log(ctx, rp, col, p, counts)
    counts.free()
    kp = p["d"] + p["oversample"]
    Om = lne.gaussian(ctx, g.n, kp, p["seed"], dtype=torch.float32, ld=(kp + 7) // 8 * 8)
    Y = lne.spmm(ctx, M, Om[:, :kp])
    M.free()
    deg = g.degrees().astype(np.int64)
    for (lo, hi), (R0, C0, W0) in refs.items():
        a, b = int(Rd[lo].item()), int(Rd[hi].item())
        np.testing.assert_array_equal((Rd[lo:hi + 1] - a).cpu().numpy(), R0)
        np.testing.assert_array_equal(Cd[a:b].cpu().numpy(), C0)
        np.testing.assert_array_equal(Wd[a:b].cpu().numpy().view(np.uint64), W0)
        keep, val = oracle.trunc_log(g, p, R0, C0, W0, row_lo=lo)
        cols = np.unique(C0)
        Omr = oracle.gaussian_omega(g.n, kp, p["seed"], rows=cols)
        idx = np.searchsorted(cols, C0)
        yd = Y[lo:hi].double().cpu().numpy()
        for r in range(hi - lo):
            s, e = R0[r], R0[r + 1]
            k = keep[s:e].astype(bool)
            v = val[s:e][k]
            O = Omr[idx[s:e][k]]
            ref = v @ O
            bar = 4 * math.sqrt(max(int(k.sum()), 1)) * 2.0 ** -24 * (np.abs(v) @ np.abs(O)) + 1e-30
            assert np.all(np.abs(yd[r] - ref) <= bar), (lo + r, np.max(np.abs(yd[r] - ref) / bar))


def test_embedding_matrix_rows_at_full_size(lne, ctx, large):
    """The matrix lne_embed factorises, built as the benchmark builds it
    (Eq. (1) fused into the aggregation, column degrees carried in the sort
    keys): on the windows its kept set is the oracle's and its FP32 values are
    the oracle's FP64 ln x rounded (within one FP32 ulp)."""
    g, p, rp, col, refs = large
    M, st = lne.sparsify_log(ctx, rp, col, p)
    Rd, Cd, Vd = M.to_torch()
    for (lo, hi), (R0, C0, W0) in refs.items():
        keep, val = oracle.trunc_log(g, p, R0, C0, W0, row_lo=lo)
        a, b = int(Rd[lo].item()), int(Rd[hi].item())
        R = (Rd[lo:hi + 1] - a).cpu().numpy()
        C = Cd[a:b].cpu().numpy()
        V = Vd[a:b].double().cpu().numpy()
        nz = V != 0
        rows = np.repeat(np.arange(hi - lo), np.diff(R))
        rows0 = np.repeat(np.arange(hi - lo), np.diff(R0))
        np.testing.assert_array_equal(rows[nz], rows0[keep])
        np.testing.assert_array_equal(C[nz], C0[keep])
        ref = val[keep]
        assert np.all(np.abs(V[nz] - ref) <= 2.0 ** -23 * np.abs(ref) + 1e-30)
    M.free()
