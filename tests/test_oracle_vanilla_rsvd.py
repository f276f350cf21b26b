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
