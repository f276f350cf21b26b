"""Parity at the benchmark's full size: the Chung-Lu graph with 10^7 vertices
and 2*10^8 edges, T = 5, s = (0.3, 0.7, 0, 0, 0), M = 4 T m, C = ln n.  The
oracle cannot walk all 4*10^9 samples, but with walk lengths r <= 2 the rows
of a vertex window only receive samples of edges incident to the window's
closed neighbourhood, which it can: on sampled windows (one of them a hub of
degree above 5,000) the count rows are bit-exact (through the row-window
entry point and through the whole-matrix sparsifier), and so are the first
rSVD product rows Y = M Omega within the FP32 accumulation bound.  The
products themselves are checked at full size on 10^4 random rows and the
largest hubs (sparse x dense rows against an FP64 product of the same rows),
the Gram matrix of the whole Y that the orthonormalisation uses against an
FP64 product of all its rows, and the propagation's graph product rows
against an FP64 product over the rows' neighbours."""
import math

import numpy as np
import pytest

import oracle
from synth import workload
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu

WINDOWS = [(123_456, 123_460), (5_000_000, 5_000_004), (9_999_990, 10_000_000)]
HUB_DEGREE = 5_000
U32 = 2.0 ** -24


def hub_window(g):
    """The vertex of degree >= HUB_DEGREE whose closed neighbourhood spans the
    fewest arcs (the cheapest hub row for the oracle)."""
    deg = np.diff(g.rowptr)
    nb_arcs = np.add.reduceat(deg[g.col].astype(np.int64), g.rowptr[:-1]) * (deg > 0) + deg
    cand = np.flatnonzero(deg >= HUB_DEGREE)
    a = int(cand[np.argmin(nb_arcs[cand])])
    return a, a + 1


@pytest.fixture(scope="module")
def large(lne, ctx):
    g, p = workload("large")
    assert np.all(np.asarray(p["s"])[2:] == 0)        # walk lengths 1 and 2 only
    rp, col = to_dev(g)
    refs = {}
    for lo, hi in WINDOWS + [hub_window(g)]:
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


def _rows_on_host(Rd, Cd, Vd, rows):
    """Rows `rows` of a device CSR as a host scipy CSR (n_sel x n_cols)."""
    import scipy.sparse as sp
    import torch
    rows_t = torch.as_tensor(rows, dtype=torch.int64, device=Rd.device)
    beg, end = Rd[rows_t], Rd[rows_t + 1]
    lens = end - beg
    idx = torch.repeat_interleave(beg - torch.cumsum(lens, 0) + lens, lens) + \
        torch.arange(int(lens.sum().item()), device=Rd.device)
    rp = np.zeros(len(rows) + 1, np.int64)
    rp[1:] = np.cumsum(lens.cpu().numpy())
    return rp, Cd[idx].cpu().numpy(), Vd[idx].double().cpu().numpy()


def test_spmm_rows_and_gram_at_full_size(lne, ctx, large):
    """The first product Y = M Omega of the embedding's matrix (built as the
    benchmark builds it) on 10^4 random rows and the four largest hubs (rows
    of about 9 10^4 nonzeros), each entry against an FP64 product of the
    same matrix row with the oracle's Omega rows within the FP32 accumulation
    bound; then the Gram matrix Y^T Y of all 10^7 rows as the eigSVD computes
    it (MFMA FP64, V diag(S^2) V^T) against an FP64 product of the whole Y on
    the host, within the worst-case FP64 summation bound n u."""
    import scipy.sparse as sp
    import torch
    g, p, rp, col, refs = large
    M, _ = lne.sparsify_log(ctx, rp, col, p)
    kp = p["d"] + p["oversample"]
    Om = lne.gaussian(ctx, g.n, kp, p["seed"], dtype=torch.float32, ld=160)
    Y = lne.spmm(ctx, M, Om)
    del Om
    Rd, Cd, Vd = M.to_torch()
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([rng.choice(g.n, 10_000, replace=False), [0, 1, 2, 3]]))
    R, C, V = _rows_on_host(Rd, Cd, Vd, rows)
    del Rd, Cd, Vd
    M.free()
    assert np.diff(R).max() > 50_000                    # a hub row among them
    cols, inv = np.unique(C, return_inverse=True)
    Omr = oracle.gaussian_omega(g.n, kp, p["seed"], rows=cols)
    A = sp.csr_matrix((V, inv, R), shape=(len(rows), len(cols)))
    ref = A @ Omr
    scale = abs(A) @ np.abs(Omr)
    nnz = np.diff(R)[:, None]
    yd = Y[torch.as_tensor(rows, device=Y.device)].double().cpu().numpy()
    bar = (4 * np.sqrt(np.maximum(nnz, 1)) + 2) * U32 * scale + 1e-30
    assert np.all(np.abs(yd - ref) <= bar), np.max(np.abs(yd - ref) / bar)
    # Gram of the whole Y, as the orthonormalisation forms it
    _, S, Vv = lne.eigsvd(ctx, Y)
    S, Vv = S.cpu().numpy(), Vv.cpu().numpy()
    G_gpu = (Vv * S ** 2) @ Vv.T
    G = np.zeros((kp, kp))
    for i in range(0, g.n, 1 << 20):
        blk = Y[i:i + (1 << 20)].double().cpu().numpy()
        G += blk.T @ blk
    err = np.linalg.norm(G_gpu - G) / np.linalg.norm(G)
    assert err <= g.n * 2.0 ** -53, err


def test_graph_spmm_rows_at_full_size(lne, ctx, large):
    """One product of the propagation recurrence, out = (1 - mu) Z - D^-1 A Z
    with Z = randn(n, d) (the device's Gaussian, regenerated on the host by
    the oracle for the rows needed), in the launch shape the propagation
    uses: 10^4 random rows and the four largest hubs against an FP64 sum over
    each row's neighbours."""
    import torch
    g, p, rp, col, refs = large
    d, mu = p["d"], p["mu"]
    Z = lne.gaussian(ctx, g.n, d, p["seed"] + 5, dtype=torch.float32, ld=d)
    out = lne.graph_spmm(ctx, rp, col, Z, 1.0 - mu, -1.0)
    rng = np.random.default_rng(12)
    rows = np.unique(np.concatenate([rng.choice(g.n, 10_000, replace=False), [0, 1, 2, 3]]))
    got = out[torch.as_tensor(rows, device=out.device)].double().cpu().numpy()
    nb = [g.col[g.rowptr[a]:g.rowptr[a + 1]] for a in rows]
    need = np.unique(np.concatenate([rows] + nb))
    Zr = oracle.gaussian_omega(g.n, d, p["seed"] + 5, rows=need)
    pos = {int(v): i for i, v in enumerate(need)}
    assert min(len(x) for x in nb) == 0                 # an isolated vertex among them
    for i, a in enumerate(rows):
        Zn = Zr[np.searchsorted(need, nb[i])]
        za = Zr[pos[int(a)]]
        # an isolated vertex has an empty row of D^-1 A
        inv = 1.0 / len(nb[i]) if len(nb[i]) else 0.0
        ref = (1.0 - mu) * za - Zn.sum(axis=0) * inv
        scale = (1.0 - mu) * np.abs(za) + np.abs(Zn).sum(axis=0) * inv
        bar = (4 * math.sqrt(len(nb[i])) + 2) * U32 * scale + 1e-30
        assert np.all(np.abs(got[i] - ref) <= bar), (a, np.max(np.abs(got[i] - ref) / bar))
