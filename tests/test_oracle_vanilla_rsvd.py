"""Pins of the vanilla randomized SVD (the comparator the paper's fast one
replaces, section 4.2) against the exact SVD and the fast randomized SVD."""
import numpy as np
import scipy.sparse as sp

import oracle



def test_vanilla_rsvd_is_exact_with_a_full_sketch():
    """With as many sketch columns as rows the vanilla randomized SVD is the
    exact truncated SVD (Q spans everything): singular values equal LAPACK's
    and U S V^T is the best rank-d approximation."""
    rng = np.random.default_rng(3)
    n, d = 40, 6
    A = rng.standard_normal((n, n))
    M = sp.csr_matrix(A + A.T)
    omega = rng.standard_normal((n, n))
    U, S, V = oracle.vanilla_rsvd(M, d, n - d, 1, omega)
    Ue, Se, Vet = np.linalg.svd(M.toarray())
    np.testing.assert_allclose(S, Se[:d], rtol=1e-12)
    best = (Ue[:, :d] * Se[:d]) @ Vet[:d]
    np.testing.assert_allclose((U * S) @ V.T, best, atol=1e-10)
    np.testing.assert_allclose(U.T @ U, np.eye(d), atol=1e-12)


def test_vanilla_and_fast_rsvd_agree_on_a_gapped_spectrum():
    """Both randomized SVDs recover the top singular values of a matrix with
    a clear spectral gap to high accuracy (they differ in how they form U)."""
    rng = np.random.default_rng(4)
    n, d = 300, 5
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.r_[np.linspace(10, 6, d), 0.01 * rng.standard_normal(n - d)]
    M = sp.csr_matrix((Qm * lam) @ Qm.T)
    omega = rng.standard_normal((n, d + 10))
    Uv, Sv, _ = oracle.vanilla_rsvd(M, d, 10, 2, omega)
    Uf, Sf, _ = oracle.fast_rsvd(M, d, 10, 2, omega)
    top = np.sort(np.abs(lam))[::-1][:d]
    np.testing.assert_allclose(Sv, top, rtol=1e-6)
    np.testing.assert_allclose(Sf, top, rtol=1e-6)
    # both U span the top eigenvectors
    for U in (Uv, Uf):
        r = Qm[:, :d] - U @ (U.T @ Qm[:, :d])
        assert np.linalg.norm(r, 2) < 1e-4


def test_sparse_sign_omega_moments_and_structure():
    """The sparse-sign test matrix: 8 signed unit entries per row (sums of
    entries keep the parity of 8), columns uniform, signs balanced, and
    E[Omega^T Omega] = n (8 / k) I (the isotropy that makes it a valid sketch)."""
    import scipy.stats
    n, k = 40000, 138
    O = oracle.sparse_sign_omega(n, k, 5)
    assert np.all(np.abs(O).sum(1) <= 8) and np.all(O.sum(1) % 2 == 0)
    assert np.all(np.abs(O).sum(1) % 2 == 0)
    occ = np.abs(O).sum(0)
    assert scipy.stats.chisquare(occ).pvalue > 1e-4
    pos, neg = (O > 0).sum(), (O < 0).sum()
    assert abs(pos - neg) < 5 * np.sqrt(pos + neg)
    G = O.T @ O / n
    # diagonal: mean 8/k, each entry's variance ~ (8/k)/n per unit
    assert np.max(np.abs(np.diag(G) - 8 / k)) < 6 * np.sqrt(8 / k / n) * 3
    off = G - np.diag(np.diag(G))
    assert np.max(np.abs(off)) < 6 * np.sqrt(8 / k / n) * np.sqrt(8 / k) * 4


def test_fast_rsvd_with_sparse_sign_omega_recovers_the_top_subspace():
    rng = np.random.default_rng(8)
    n, d = 400, 5
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.r_[np.linspace(10, 6, d), 0.01 * rng.standard_normal(n - d)]
    M = sp.csr_matrix((Qm * lam) @ Qm.T)
    omega = oracle.sparse_sign_omega(n, d + 10, 3)
    U, S, _ = oracle.fast_rsvd(M, d, 10, 2, omega)
    np.testing.assert_allclose(S, np.sort(np.abs(lam))[::-1][:d], rtol=1e-6)
    r = Qm[:, :d] - U @ (U.T @ Qm[:, :d])
    assert np.linalg.norm(r, 2) < 1e-4
