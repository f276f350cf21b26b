"""GPU SpMM, eigSVD, CholeskyQR2 orthonormaliser, fast randomized SVD and
spectral propagation vs the oracle and LAPACK."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synth import workload
from tests import graphs_small as gs
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24
UBF = 2.0 ** -8


def principal_angle(A, B):
    """Largest principal angle between span(A) and span(B), as
    arcsin ||(I - Qa Qa^T) Qb||_2 (accurate for small angles)."""
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    r = qb - qa @ (qa.T @ qb)
    return float(np.arcsin(min(1.0, np.linalg.norm(r, 2))))


def procrustes_err(X, Xref):
    U, _, Vt = np.linalg.svd(X.T @ Xref)
    return float(np.linalg.norm(X @ (U @ Vt) - Xref) / np.linalg.norm(Xref))


@pytest.fixture(scope="module")
def tiny(lne, ctx):
    g, p = workload("tiny")
    rp, col = to_dev(g)
    st = oracle.embed(g, p, return_stages=True)
    return g, p, rp, col, st


def _rand_y(n, k, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, k)))
    Q2, _ = np.linalg.qr(rng.standard_normal((k, k)))
    return (Q1 * np.logspace(0, -math.log10(cond), k)) @ Q2


# 138 and 139: the last width whose Gram fits the eigensolver's LDS variant
# and the first that takes the global-memory one; 288: the widest accepted
@pytest.mark.parametrize("k", [5, 42, 138, 139, 140, 272, 288])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_eigsvd_vs_lapack(lne, ctx, k, dtype):
    import torch
    n = 3000
    Y = _rand_y(n, k, seed=k, cond=10.0 if dtype == "bf16" else 1e3)
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    ld = (k + 7) // 8 * 8
    Yd = torch.zeros((n, ld), dtype=tdt, device="cuda")
    Yd[:, :k] = torch.from_numpy(Y).to(tdt)
    Yq = Yd[:, :k].double().cpu().numpy()         # the values the GPU sees
    U, S, V = lne.eigsvd(ctx, Yd[:, :k])
    S2 = np.linalg.svd(Yq, compute_uv=False)
    tol = {"f64": 1e-11, "f32": 1e-10, "bf16": 4 * UBF}[dtype]
    np.testing.assert_allclose(S.cpu().numpy(), S2, rtol=tol * 10, atol=tol * S2[0])
    Un = U.double().cpu().numpy()
    Vn = V.cpu().numpy()
    recon = (Un * S.cpu().numpy()) @ Vn.T
    rt = {"f64": 1e-12, "f32": 1e-6, "bf16": 2e-2}[dtype]
    assert np.linalg.norm(recon - Yq) <= rt * np.linalg.norm(Yq)
    np.testing.assert_allclose(Vn.T @ Vn, np.eye(k), atol=1e-12)


def _structured_y(n, k, kind, seed):
    """Inputs whose Gram matrices drive the eigen-solver's deflation: exactly
    repeated singular values, a rank-deficient Y (zero eigenvalues) and
    orthogonal columns (an already diagonal Gram, no coupling anywhere)."""
    rng = np.random.default_rng(seed)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, k)))
    if kind == "diagonal":
        return Q1 * np.linspace(3.0, 1.0, k)
    Q2, _ = np.linalg.qr(rng.standard_normal((k, k)))
    if kind == "clustered":
        s = np.repeat([10.0, 3.0, 1.0], (k + 2) // 3)[:k]
    else:   # rank-deficient: a third of the directions carry the data
        s = np.where(np.arange(k) < max(1, k // 3), np.linspace(5.0, 1.0, k), 0.0)
    return (Q1 * s) @ Q2


# 31 / 32 / 33 straddle the size from which the tridiagonal matrix is torn in
# two and merged; 138 and 266 are the embedding and precision widths
@pytest.mark.parametrize("k", [31, 32, 33, 138, 266])
@pytest.mark.parametrize("kind", ["clustered", "rankdef", "diagonal"])
def test_eigsvd_structured_spectra(lne, ctx, k, kind):
    import torch
    n = 2000
    Y = _structured_y(n, k, kind, seed=k)
    Yd = torch.from_numpy(Y).cuda()
    U, S, V = lne.eigsvd(ctx, Yd)
    S = S.cpu().numpy()
    Vn = V.cpu().numpy()
    S2 = np.linalg.svd(Y, compute_uv=False)
    # eigenvalues of the Gram to an absolute 1e-13 of the largest, so the
    # singular values to that over 2 s_i, and exact zeros to sqrt of it
    lam, lam2 = S ** 2, S2 ** 2
    assert np.max(np.abs(lam - lam2)) <= 1e-13 * lam2[0] * k
    np.testing.assert_allclose(Vn.T @ Vn, np.eye(k), atol=1e-12)
    # V diagonalises the Gram: V^T G V = diag(S^2) to rounding
    G = Y.T @ Y
    off = Vn.T @ G @ Vn - np.diag(lam)
    assert np.max(np.abs(off)) <= 1e-12 * lam2[0]
    Un = U.cpu().numpy()
    keep = S > k * 2.220446049250313e-16 * S[0]
    assert np.linalg.norm((Un[:, keep] * S[keep]) - Y @ Vn[:, keep]) <= 1e-12 * np.linalg.norm(Y)
    assert np.all(Un[:, ~keep] == 0.0)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("k", [42, 138])
def test_orthonormalize(lne, ctx, dtype, k):
    import torch
    n = 5000
    Y = _rand_y(n, k, seed=3, cond=1e4)
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dtype]
    ld = (k + 7) // 8 * 8
    Yd = torch.zeros((n, ld), dtype=tdt, device="cuda")
    Yd[:, :k] = torch.from_numpy(Y).to(tdt)
    Yq = Yd[:, :k].double().cpu().numpy()
    lne.orthonormalize(ctx, Yd[:, :k])
    Q = Yd[:, :k].double().cpu().numpy()
    tol = {"f64": 1e-13, "f32": 3e-6, "bf16": 6e-2}[dtype]
    assert np.max(np.abs(Q.T @ Q - np.eye(k))) < tol * math.sqrt(k)
    assert principal_angle(Q, Yq) < {"f64": 1e-8, "f32": 1e-2, "bf16": 0.5}[dtype]


def test_orthonormalize_ill_conditioned_takes_shift(lne, ctx):
    import torch
    n, k = 4000, 40
    Y = _rand_y(n, k, seed=9, cond=1e12)
    Yd = torch.from_numpy(Y).cuda()
    lne.orthonormalize(ctx, Yd)
    Q = Yd.cpu().numpy()
    assert np.max(np.abs(Q.T @ Q - np.eye(k))) < 1e-12


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_spmm_vs_scipy(lne, ctx, tiny, prec):
    import torch
    g, p, rp, col, st = tiny
    pp = dict(p, precision=prec)
    counts, _ = lne.sparsify(ctx, rp, col, pp)
    M = lne.trunc_log(ctx, rp, col, pp, counts)
    R, C, V = (x.cpu() for x in M.to_torch())
    A = sp.csr_matrix((V.double().numpy(), C.numpy(), R.numpy()), shape=(g.n, g.n))
    # widths with no tail, a fused tail, k below one vector and tails that
    # take a launch of their own
    for k in (1, 3, 8, 42, 138, 200, 300):
        rng = np.random.default_rng(k)
        X = rng.standard_normal((g.n, k))
        tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[prec]
        ld = (k + 7) // 8 * 8
        Xd = torch.zeros((g.n, ld), dtype=tdt, device="cuda")
        Xd[:, :k] = torch.from_numpy(X).to(tdt)
        Y = lne.spmm(ctx, M, Xd[:, :k]).double().cpu().numpy()
        ref = A @ Xd[:, :k].double().cpu().numpy()
        scale = np.abs(A) @ np.abs(Xd[:, :k].double().cpu().numpy())
        u = {"f64": U64, "f32": U32, "bf16": UBF}[prec]
        assert np.all(np.abs(Y - ref) <= 4 * np.sqrt(A.getnnz(1).max()) * u * scale + 1e-300)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_spmm_launch_shapes_give_identical_results(lne, ctx, tiny, tmp_path, monkeypatch, prec):
    """Every unroll depth the tuner may pick computes the same bits: each lane
    group accumulates its nonzeros in row order whatever the depth.  A fresh
    context reads the choice from the tuning cache file."""
    import torch
    g, p, rp, col, st = tiny
    pp = dict(p, precision=prec)
    counts, _ = lne.sparsify(ctx, rp, col, pp)
    M = lne.trunc_log(ctx, rp, col, pp, counts)
    tdt = torch.float64 if prec == "f64" else torch.float32
    code = 0 if prec == "f64" else 1
    outs = []
    for v in range(4):
        for k in (8, 136):
            path = tmp_path / f"tune_{v}_{k}.jsonl"
            key = (f'"op": "spmm", "n": {g.n}, "nnz_class": {math.floor(4 * math.log2(M.nnz))}, '
                   f'"k": {k}, "dtype": {code}')
            gkey = (f'"op": "graph_spmm", "n": {g.n}, "nnz_class": '
                    f'{math.floor(4 * math.log2(g.n_arcs))}, "k": {k}, "dtype": {code}')
            path.write_text(f'{{{key}, "variant": {v}, "ms": []}}\n'
                            f'{{{gkey}, "variant": {v}, "ms": []}}\n')
            monkeypatch.setenv("LNE_TUNE_CACHE", str(path))
            c2 = lne.Context()
            X = torch.from_numpy(np.random.default_rng(k).standard_normal((g.n, k))).to(tdt).cuda()
            Y = lne.spmm(c2, M, X)
            Z = lne.propagate(c2, rp, col, dict(pp, flags=lne.FLAG_NO_FINAL_EIGSVD, d=k), X)
            outs.append((k, Y.cpu().numpy(), Z.cpu().numpy()))
            c2.close()
            assert path.read_text().count("\n") == 2          # nothing re-tuned
    for k in (8, 136):
        same = [o for o in outs if o[0] == k]
        for o in same[1:]:
            np.testing.assert_array_equal(o[1], same[0][1])
            np.testing.assert_array_equal(o[2], same[0][2])


def test_rsvd_matches_oracle_f64(lne, ctx, tiny):
    g, p, rp, col, st = tiny
    counts, _ = lne.sparsify(ctx, rp, col, p)
    M = lne.trunc_log(ctx, rp, col, p, counts)
    U, S, V, X0 = (x.cpu().numpy() for x in lne.rsvd(ctx, M, p))
    Sref = st["S"]
    kp = p["d"] + p["oversample"]
    # full spectrum of the basis, for the gap at d
    gap = (Sref[-2] - Sref[-1]) / Sref[0] if len(Sref) > 1 else 1.0
    tol = 100 * math.sqrt(kp) * U64 / max(gap, 1e-3)
    np.testing.assert_allclose(S, Sref, rtol=10 * math.sqrt(kp) * U64 * Sref[0] / Sref.min() + 1e-12)
    assert principal_angle(U, st["U"]) < max(tol, 1e-9)
    assert procrustes_err(X0, st["X0"]) < max(tol, 1e-9)
    assert procrustes_err(V, st["V"]) < max(tol, 1e-9)


@pytest.mark.parametrize("q", [1, 2])
def test_rsvd_vanilla_matches_oracle_f64(lne, ctx, tiny, q):
    """The vanilla randomized SVD (flag) against the oracle's HMT version:
    U = Q U_B from the SVD of B = Q^T M."""
    g, p, rp, col, st = tiny
    pp = dict(p, q=q, flags=lne.FLAG_VANILLA_RSVD)
    counts, _ = lne.sparsify(ctx, rp, col, pp)
    M = lne.trunc_log(ctx, rp, col, pp, counts)
    U, S, V, X0 = (x.cpu().numpy() for x in lne.rsvd(ctx, M, pp))
    kp = p["d"] + p["oversample"]
    omega = oracle.gaussian_omega(g.n, kp, p["seed"])
    Uo, So, Vo = oracle.vanilla_rsvd(st["M"], p["d"], p["oversample"], q, omega)
    gap = (So[-2] - So[-1]) / So[0]
    tol = 100 * math.sqrt(kp) * U64 / max(gap, 1e-3)
    np.testing.assert_allclose(S, So, rtol=10 * math.sqrt(kp) * U64 * So[0] / So.min() + 1e-12)
    assert principal_angle(U, Uo) < max(tol, 1e-9)
    assert procrustes_err(V, Vo) < max(tol, 1e-9)
    assert procrustes_err(X0, Uo * np.sqrt(So)) < max(tol, 1e-9)
    # the fast randomized SVD of the same run takes U from M Q instead
    Uf = lne.rsvd(ctx, M, dict(p, q=q))[0].cpu().numpy()
    assert principal_angle(Uf, U) > 10 * max(tol, 1e-9)


def test_embed_vanilla_matches_oracle(lne, ctx, tiny):
    g, p, rp, col, st = tiny
    pp = dict(p, flags=lne.FLAG_VANILLA_RSVD)
    X, _ = lne.embed(ctx, rp, col, pp)
    ref = oracle.embed(g, pp)
    assert procrustes_err(X.cpu().numpy(), ref) < 1e-8


def _dense_omega(om, k):
    om = om.astype(np.int64)
    out = np.zeros((om.shape[0], k))
    c = np.abs(om) - 1
    np.add.at(out, (np.repeat(np.arange(om.shape[0]), om.shape[1]), c.ravel()),
              np.sign(om).ravel().astype(np.float64))
    return out


def test_sparse_omega_matches_oracle(lne, ctx):
    for n, k, seed in ((1000, 42, 1), (5003, 138, 9)):
        om = lne.sparse_omega(ctx, n, k, seed).cpu().numpy()
        np.testing.assert_array_equal(_dense_omega(om, k), oracle.sparse_sign_omega(n, k, seed))


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_spmm_sparse_omega_vs_scipy(lne, ctx, tiny, prec):
    import torch
    g, p, rp, col, st = tiny
    pp = dict(p, precision=prec)
    counts, _ = lne.sparsify(ctx, rp, col, pp)
    M = lne.trunc_log(ctx, rp, col, pp, counts)
    R, C, V = (x.cpu() for x in M.to_torch())
    A = sp.csr_matrix((V.double().numpy(), C.numpy(), R.numpy()), shape=(g.n, g.n))
    for k in (42, 138):
        om = lne.sparse_omega(ctx, g.n, k, 4)
        tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[prec]
        Y = lne.spmm_sparse_omega(ctx, M, om, k, tdt).double().cpu().numpy()
        O = _dense_omega(om.cpu().numpy(), k)
        ref = A @ O
        scale = np.abs(A) @ np.abs(O)
        u = {"f64": U64, "f32": U32, "bf16": UBF}[prec]
        assert np.all(np.abs(Y - ref) <= 4 * np.sqrt(A.getnnz(1).max() * 8) * u * scale + 1e-300)


def test_rsvd_and_embed_with_sparse_omega_match_oracle(lne, ctx, tiny):
    g, p, rp, col, st = tiny
    pp = dict(p, flags=lne.FLAG_SPARSE_OMEGA)
    counts, _ = lne.sparsify(ctx, rp, col, pp)
    M = lne.trunc_log(ctx, rp, col, pp, counts)
    U, S, V, X0 = (x.cpu().numpy() for x in lne.rsvd(ctx, M, pp))
    kp = p["d"] + p["oversample"]
    omega = oracle.sparse_sign_omega(g.n, kp, p["seed"])
    Uo, So, Vo = oracle.fast_rsvd(st["M"], p["d"], p["oversample"], p["q"], omega)
    gap = (So[-2] - So[-1]) / So[0]
    tol = 100 * math.sqrt(kp) * U64 / max(gap, 1e-3)
    np.testing.assert_allclose(S, So, rtol=10 * math.sqrt(kp) * U64 * So[0] / So.min() + 1e-12)
    assert principal_angle(U, Uo) < max(tol, 1e-9)
    assert procrustes_err(V, Vo) < max(tol, 1e-9)
    X, _ = lne.embed(ctx, rp, col, pp)
    assert procrustes_err(X.cpu().numpy(), oracle.embed(g, pp)) < 1e-8


@pytest.mark.parametrize("k,theta,mu", [(10, 0.5, 0.2), (3, 1.0, 0.4), (1, 0.3, 0.0)])
def test_propagate_filter_matches_oracle(lne, ctx, tiny, k, theta, mu):
    import torch
    g, p, rp, col, st = tiny
    X0 = st["X0"]
    pp = dict(p, cheb_k=k, theta=theta, mu=mu, flags=lne.FLAG_NO_FINAL_EIGSVD)
    Xsp = lne.propagate(ctx, rp, col, pp, torch.from_numpy(X0).cuda()).cpu().numpy()
    ref = oracle.propagate(g, X0, k, theta, mu)
    assert np.max(np.abs(Xsp - ref)) <= 1e-12 * np.max(np.abs(X0)) * (2 * k + 1)


@pytest.mark.parametrize("d", [3, 42, 138, 200])
def test_propagate_filter_widths(lne, ctx, tiny, d):
    """Operand widths with a fused tail, a tail of its own launch and one
    below a single vector give the oracle's filter."""
    import torch
    g, p, rp, col, st = tiny
    X0 = np.random.default_rng(d).standard_normal((g.n, d))
    pp = dict(p, d=d, cheb_k=4, theta=0.7, mu=0.1, flags=lne.FLAG_NO_FINAL_EIGSVD)
    for prec, tol in (("f64", 1e-12), ("f32", 1e-5)):
        tdt = torch.float64 if prec == "f64" else torch.float32
        X0d = torch.from_numpy(X0).to(tdt).cuda()
        Xsp = lne.propagate(ctx, rp, col, dict(pp, precision=prec), X0d).double().cpu().numpy()
        ref = oracle.propagate(g, X0d.double().cpu().numpy(), 4, 0.7, 0.1)
        assert np.max(np.abs(Xsp - ref)) <= tol * np.max(np.abs(X0)) * 9


def test_propagate_final_embedding(lne, ctx, tiny):
    import torch
    g, p, rp, col, st = tiny
    X = lne.propagate(ctx, rp, col, p, torch.from_numpy(st["X0"]).cuda()).cpu().numpy()
    assert procrustes_err(X, st["X"]) < 1e-9


def test_propagate_off_is_identity(lne, ctx, tiny):
    import torch
    g, p, rp, col, st = tiny
    X0 = torch.from_numpy(st["X0"]).cuda()
    for pp in (dict(p, cheb_k=0), dict(p, theta=0.0)):
        assert bool((lne.propagate(ctx, rp, col, pp, X0) == X0).all())


def test_embed_tiny_matches_oracle(lne, ctx, tiny):
    g, p, rp, col, st = tiny
    X, stats = lne.embed(ctx, rp, col, p)
    X = X.cpu().numpy()
    assert stats["nnz_log"] == st["M"].nnz
    assert principal_angle(X, st["X"]) < 1e-8
    assert procrustes_err(X, st["X"]) < 1e-8


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_embed_degenerate_graphs_give_zero(lne, ctx, prec):
    """No edges (no samples at all) and a sparsifier truncated to nothing
    (K4,4 at b = 2): the zero matrix, whose embedding is exactly zero, as the
    oracle's."""
    g = gs.from_edges(60, [])
    p = dict(gs.params(T=3, M_per_m=10, m=1), d=4, oversample=2, q=1, cheb_k=3, theta=0.5,
             mu=0.2, precision=prec)
    rp, col = to_dev(g)
    X, st = lne.embed(ctx, rp, col, p)
    assert st["accepted"] == 0 and st["nnz_log"] == 0
    assert X.shape == (60, 4) and bool((X == 0).all())
    k44 = gs.from_edges(8, [(i, j) for i in range(4) for j in range(4, 8)])
    p = gs.params(T=1, s=[1.0], M_per_m=5, C=None, m=k44.m, b=2)
    p.update(d=2, oversample=2, q=2, cheb_k=2, theta=0.5, mu=0.2, precision=prec)
    rp, col = to_dev(k44)
    X, st = lne.embed(ctx, rp, col, p)
    assert st["accepted"] > 0 and st["nnz_log"] == 0
    assert bool((X == 0).all())
    assert np.all(oracle.embed(k44, p) == 0.0)


def test_embed_keeps_few_dropped_pairs_as_explicit_zeros(lne, ctx):
    """With few pairs dropped by Eq. (1)'s truncation the embedding path keeps
    them as explicit zeros instead of compacting; the embedding and the kept
    count still match the oracle."""
    g, p = workload("tiny")
    p = dict(p, M=3 * p["T"] * g.m, seed=11)
    R, C, W, _, _ = oracle.count_csr(g, p)
    keep, _ = oracle.trunc_log(g, p, R, C, W)
    dropped = len(keep) - int(keep.sum())
    assert 0 < dropped < len(keep) / 32
    rp, col = to_dev(g)
    ref = oracle.embed(g, p, return_stages=True)
    X, stats = lne.embed(ctx, rp, col, p)
    assert stats["nnz_log"] == ref["M"].nnz == int(keep.sum())
    assert stats["nnz_counts"] == len(keep)
    assert procrustes_err(X.cpu().numpy(), ref["X"]) < 1e-8


def test_embed_hub_above_16_bit_degree(lne, ctx):
    """A hub of degree above 65535 (degree products past 2^32 in Eq. (1)'s
    keep test): the pairs and the kept count match the oracle exactly."""
    from synth.graphs import Graph, _csr_from_pairs
    n = 70001
    leaves = np.arange(1, n, dtype=np.int64)
    a = np.concatenate([np.zeros(n - 1, np.int64), leaves[:-1]])    # star + path
    b = np.concatenate([leaves, leaves[1:]])
    rowptr, col = _csr_from_pairs(a, b, n, "cpu")
    g = Graph(n, rowptr, col, None, "star-path")
    assert g.degrees().max() > 65535
    _, p = workload("tiny")
    p = dict(p, M=p["T"] * g.m, seed=5, d=8, oversample=4)
    R, C, W, _, _ = oracle.count_csr(g, p)
    keep, _ = oracle.trunc_log(g, p, R, C, W)
    rp, cold = to_dev(g)
    _, stats = lne.embed(ctx, rp, cold, p)
    assert stats["nnz_counts"] == len(keep)
    assert stats["nnz_log"] == int(keep.sum())
