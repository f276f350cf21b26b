"""Error bars of the FP32 paths against the FP64 oracle, derived from the
oracle's own quantities (test infrastructure: nothing here comes from the GPU).

Notation: u the unit roundoff of the computing type, k' = d + oversample,
s_1 >= s_2 >= ... the singular values of the last power step of the fast
randomized SVD (section 4.2), F the propagation operator of section 4.3 on
the input graph, X_sp = F X0, X = U_p S_p^(1/2) its final scaling.

* rSVD: every stored n x k' block is rounded entry by entry (relative u), so
  the products the randomized SVD factorises move by at most sqrt(k') u s_1 in
  the 2-norm; with a few such roundings per power step the perturbation is
  e = 4 sqrt(k') u s_1.  X0 = U_d S_d^(1/2) then moves (up to an orthogonal
  alignment) by at most e sqrt(d) / (2 sqrt(s_d)) inside the top-d space (a
  rotation between directions i, j moves X0 by e / (sqrt(s_i) + sqrt(s_j)))
  plus e sqrt(s_d) / (s_d - s_d+1) across the boundary at d.
* Propagation: F = D^-1 A (I - g_k(L)) is a polynomial in the walk matrix,
  so F^T = D F D^-1 and |F|_2 follows from a power iteration on F^T F with the
  oracle's own propagate.  Rounding is bounded in the D^(1/2)-weighted norm,
  where the walk matrix is a contraction and every Chebyshev term T_n is
  bounded by one: a graph product out = a Z + b D^-1 A Z + ... adds at most
  g = (4 sqrt(d_max) + 3) u of its operands, so a recurrence step (B = L - mu
  I applied twice, |B| <= 2, then the three-term update) adds at most 7 g;
  the recurrence carries an error made at step j to step n with a factor of
  at most n - j + 1 (Chebyshev polynomials of the second kind), so the
  accumulated sum_n c_n T_n is off by at most 7 g sum_n |c_n| (n+1)(n+2)/2,
  its own accumulation by g sum_n |c_n|, and the last product D^-1 A (X0 -
  sum) by 2 g.  Back in the 2-norm this costs kappa_D = sqrt(d_max / d_min):
  e_prop = kappa_D g (7 sum_n |c_n| (n+1)(n+2)/2 + sum_n |c_n| + 2)
           |X0| / |X_sp|.
* Final scaling: a perturbation E of X_sp moves X = U_p S_p^(1/2) by at most
  |E| / sqrt(s_min(X_sp)) (along the smallest singular direction), i.e. by
  sqrt(sum s^2) / sqrt(s_min sum s) relative to |X|_F per unit relative
  change of X_sp.
"""
import math

import numpy as np

import oracle


def rsvd_perturbation(S, kp, u):
    """e / s_1 = 4 sqrt(k') u."""
    return 4 * math.sqrt(kp) * u


def x0_bar(S, d, kp, u):
    """Relative Procrustes bar of X0 = U_d S_d^(1/2)."""
    e = rsvd_perturbation(S, kp, u) * S[0]
    gap = S[d - 1] - S[d]
    err = e * math.sqrt(d) / (2 * math.sqrt(S[d - 1])) + e * math.sqrt(S[d - 1]) / gap
    return err / math.sqrt(np.sum(S[:d]))


def propagation_norm(g, k, theta, mu, iters=60, seed=0):
    """|F|_2 of X -> D^-1 A (X - g_k(L) X) by power iteration on F^T F, with
    F^T x = D F (D^-1 x) (zero on isolated vertices, whose rows and columns of
    F vanish)."""
    deg = oracle.degrees(g).astype(np.float64)
    inv = np.where(deg > 0, 1.0 / np.where(deg > 0, deg, 1.0), 0.0)
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((g.n, 1))
    lam = 0.0
    for _ in range(iters):
        x /= np.linalg.norm(x)
        y = oracle.propagate(g, x, k, theta, mu)
        z = deg[:, None] * oracle.propagate(g, inv[:, None] * y, k, theta, mu)
        lam = float(np.linalg.norm(z))
        x = z
    return math.sqrt(lam) * 1.01          # a margin for the unconverged tail


def propagation_rounding(g, X0, Xsp, k, theta, u):
    deg = oracle.degrees(g).astype(np.float64)
    pos = deg[deg > 0]
    kappa_d = math.sqrt(pos.max() / pos.min())
    c = np.abs(oracle.cheb_coeffs(theta, k))
    n = np.arange(k + 1)
    growth = 7 * float(np.sum(c * (n + 1) * (n + 2) / 2)) + float(np.sum(c)) + 2
    gamma = (4 * math.sqrt(pos.max()) + 3) * u
    return kappa_d * gamma * growth * np.linalg.norm(X0) / np.linalg.norm(Xsp)


def final_scaling(Xsp):
    s = np.linalg.svd(Xsp, compute_uv=False)
    return math.sqrt(np.sum(s ** 2)) / math.sqrt(s.min() * np.sum(s))


def embedding_bar(g, X0, Xsp, S, d, kp, trial, u=2.0 ** -24):
    """Relative Procrustes bar of the FP32 embedding: X0's bar alone when
    propagation is off, else final_scaling * (|F|_2 |X0| / |X_sp| * e0 +
    e_prop)."""
    e0 = x0_bar(S, d, kp, u)
    if Xsp is None:
        return e0
    k, theta, mu = trial["k"], trial["theta"], trial["mu"]
    amp = propagation_norm(g, k, theta, mu) * np.linalg.norm(X0) / np.linalg.norm(Xsp)
    return final_scaling(Xsp) * (amp * e0 + propagation_rounding(g, X0, Xsp, k, theta, u))
