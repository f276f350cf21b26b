"""Pins of the oracle's linear algebra: eigSVD and the fast randomized SVD
(section 4.2, Eq. (2)) against LAPACK routines, exact low-rank recovery and
the error bound; spectral propagation (section 4.3) against the closed form
through a dense eigendecomposition and the filter it expands."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
from synth import sbm
from tests import graphs_small as gs


def principal_angle(A, B):
    """Largest principal angle between span(A) and span(B), as
    arcsin ||(I - Qa Qa^T) Qb||_2 (accurate for small angles)."""
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    r = qb - qa @ (qa.T @ qb)
    return float(np.arcsin(min(1.0, np.linalg.norm(r, 2))))


def rand_sym(n, spectrum, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * spectrum) @ Q.T, Q


def test_eigsvd_matches_lapack_svd():
    rng = np.random.default_rng(0)
    Y = rng.standard_normal((300, 20)) @ np.diag(np.logspace(0, -3, 20))
    U, S, V = oracle.eigsvd(Y)
    U2, S2, Vt2 = np.linalg.svd(Y, full_matrices=False)
    np.testing.assert_allclose(S, S2, rtol=1e-10)
    np.testing.assert_allclose(U.T @ U, np.eye(20), atol=1e-9)
    np.testing.assert_allclose((U * S) @ V.T, Y, atol=1e-12)
    # columns agree up to sign
    np.testing.assert_allclose(np.abs(np.sum(U * U2, 0)), 1.0, atol=1e-8)


def test_eigsvd_rank_deficient_columns_are_zero():
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((100, 3)) @ rng.standard_normal((3, 6))
    U, S, V = oracle.eigsvd(Y)
    assert np.all(S[3:] == 0) and np.all(U[:, 3:] == 0)
    np.testing.assert_allclose((U * S) @ V.T, Y, atol=1e-10)


def test_fast_rsvd_recovers_exact_low_rank():
    spec = np.zeros(200)
    spec[:6] = [9.0, -7.0, 5.0, 4.0, -2.0, 1.0]
    M, Q = rand_sym(200, spec, 2)
    omega = oracle.gaussian_omega(200, 10, seed=3)
    U, S, V = oracle.fast_rsvd(M, 8, 2, 1, omega)
    np.testing.assert_allclose(S[:6], [9, 7, 5, 4, 2, 1], rtol=1e-10)
    np.testing.assert_allclose((U * S) @ V.T, M, atol=1e-10)


def test_fast_rsvd_matches_dense_top_d():
    spec = np.concatenate([[10, 9, 8, 7], 0.5 * np.ones(296)]) * np.where(np.arange(300) % 2, -1, 1)
    M, Q = rand_sym(300, spec, 4)
    omega = oracle.gaussian_omega(300, 14, seed=5)
    U, S, V = oracle.fast_rsvd(M, 4, 10, 6, omega)
    np.testing.assert_allclose(S, [10, 9, 8, 7], rtol=1e-6)
    assert principal_angle(U, Q[:, :4]) < 1e-5


def test_orthonormaliser_choice_does_not_change_result():
    """eigSVD and Householder QR span the same subspace, and the final
    (U, S, T V) depends only on that span."""
    g = sbm([40, 40, 40], 0.3, 0.02, seed=1)
    p = gs.params(T=3, s=[0.3, 0.4, 0.3], M_per_m=200, C=math.log(g.n), m=g.m, seed=2)
    M = oracle.netmf_sparse(g, p)
    omega = oracle.gaussian_omega(g.n, 12, seed=7)
    for q in (1, 3):
        U1, S1, V1 = oracle.fast_rsvd(M, 6, 6, q, omega, orth="eigsvd")
        U2, S2, V2 = oracle.fast_rsvd(M, 6, 6, q, omega, orth="householder")
        np.testing.assert_allclose(S1, S2, rtol=1e-10)
        np.testing.assert_allclose(np.abs(np.sum(U1 * U2, 0)), 1, atol=1e-8)
        np.testing.assert_allclose((U1 * S1) @ V1.T, (U2 * S2) @ V2.T, atol=1e-9)


def test_error_bound_eq2():
    """E||M - M Q Q^T||_2 <= [1 + sqrt(d/(s-1)) + e sqrt(d+s)/s sqrt(n-d)]^(1/(q+1)) sigma_{d+1}
    averaged over 20 Gaussian test matrices."""
    n, d, s = 200, 5, 5
    spec = np.concatenate([np.linspace(10, 6, d), np.geomspace(3, 0.01, n - d)])
    M, _ = rand_sym(n, spec, 6)
    for q in (1, 2):
        errs = []
        for seed in range(20):
            omega = oracle.gaussian_omega(n, d + s, seed=100 + seed)
            Y = M @ omega
            Q = oracle.eigsvd(Y)[0]
            for _ in range(q):
                Q = oracle.eigsvd(M @ Q)[0]
            errs.append(np.linalg.norm(M - M @ Q @ Q.T, 2))
        bound = (1 + math.sqrt(d / (s - 1)) + math.e * math.sqrt(d + s) / s * math.sqrt(n - d)) ** (1 / (q + 1)) * spec[d]
        assert np.mean(errs) <= bound
        # Q has d + s columns, so no basis can do better than sigma_{d+s+1}
        assert np.mean(errs) >= spec[d + s] * (1 - 1e-9)


def test_q_zero_rejected():
    with pytest.raises(ValueError):
        oracle.fast_rsvd(np.eye(4), 1, 1, 0, np.ones((4, 2)))


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("theta,mu,k", [(0.5, 0.2, 10), (1.0, 0.0, 4), (0.9707, 0.1216, 20)])
def test_chebyshev_coefficients_expand_the_filter(theta, mu, k):
    """sum_n c_n T_n(x(lambda)) reproduces exp(-theta/2 ((lambda - mu)^2 - 1))
    on lambda in [0, 2] within the Bessel tail bound."""
    lam = np.linspace(0, 2, 401)
    x = 0.5 * (lam - mu) ** 2 - 1
    assert np.all(np.abs(x) <= 1 + 1e-12)
    approx = np.polynomial.chebyshev.chebval(x, oracle.cheb_coeffs(theta, k))
    exact = np.exp(-0.5 * theta * ((lam - mu) ** 2 - 1))
    assert np.max(np.abs(approx - exact)) <= oracle.bessel_tail_bound(theta, k) + 1e-14


def test_propagation_recurrence_matches_dense_closed_form():
    g = gs.kite()
    rng = np.random.default_rng(0)
    X0 = rng.standard_normal((g.n, 3))
    for theta, mu, k in [(0.5, 0.2, 10), (1.0, 0.4, 3), (0.3, 0.0, 1)]:
        a = oracle.propagate(g, X0, k, theta, mu)
        b = oracle.propagate_dense(g, X0, k, theta, mu)
        np.testing.assert_allclose(a, b, atol=1e-12)


def test_propagation_converges_to_filter():
    g = sbm([20, 20], 0.4, 0.05, seed=3)
    rng = np.random.default_rng(1)
    X0 = rng.standard_normal((g.n, 4))
    theta, mu = 0.8, 0.3
    exact = oracle.propagate_dense(g, X0, 0, theta, mu, exact=True)
    for k in (2, 6, 12):
        a = oracle.propagate(g, X0, k, theta, mu)
        deg = g.degrees().astype(float)
        # the filter acts as D^-1/2 V g V^T D^1/2: scale the sup bound by the
        # degree spread; the final D^-1 A has norm <= 1 in that metric
        bound = oracle.bessel_tail_bound(theta, k) * math.sqrt(deg.max() / deg.min()) * np.abs(X0).sum(0).max()
        assert np.max(np.abs(a - exact)) <= bound + 1e-12


def test_propagation_off_returns_input():
    g = gs.kite()
    X0 = np.arange(14.0).reshape(7, 2)
    np.testing.assert_array_equal(oracle.propagate(g, X0, 0, 0.5, 0.2), X0)
    np.testing.assert_array_equal(oracle.propagate(g, X0, 5, 0.0, 0.2), X0)


def test_embed_pipeline_shapes_and_scale():
    from synth import workload
    g, p = workload("tiny")
    st = oracle.embed(g, p, return_stages=True)
    assert st["X"].shape == (g.n, p["d"])
    # X0 = U S^1/2: X0^T X0 = diag(S)
    np.testing.assert_allclose(st["X0"].T @ st["X0"], np.diag(st["S"]), atol=1e-8 * st["S"][0])
    # final X = U_p S_p^1/2 with orthonormal U_p: X^T X is diagonal
    G = st["X"].T @ st["X"]
    assert np.max(np.abs(G - np.diag(np.diag(G)))) < 1e-8 * np.max(np.diag(G))
    assert sp.issparse(st["M"])
    # the sparsified matrix is symmetric
    assert abs(st["M"] - st["M"].T).max() == 0


def test_degenerate_graphs_embed_to_zero():
    """A graph without edges has no samples and an all-truncated sparsifier
    (K4,4 at b = 2: every x_ab is exactly 1) is the zero matrix; its SVD has
    only zero singular values, so the embedding U sqrt(S) and its
    propagation are exactly zero (not NaN)."""
    from tests import graphs_small as gs
    g = gs.from_edges(60, [])
    X = oracle.embed(g, dict(gs.params(T=3, M_per_m=10, m=1), d=4, oversample=2, q=1,
                             cheb_k=3, theta=0.5, mu=0.2, precision="f64"))
    assert X.shape == (60, 4) and np.all(X == 0.0)
    k44 = gs.from_edges(8, [(i, j) for i in range(4) for j in range(4, 8)])
    p = gs.params(T=1, s=[1.0], M_per_m=5, C=None, m=k44.m, b=2)
    p.update(d=2, oversample=2, q=1, cheb_k=2, theta=0.5, mu=0.2, precision="f64")
    st = oracle.embed(k44, p, return_stages=True)
    assert st["M"].nnz == 0 and np.all(st["X"] == 0.0)
