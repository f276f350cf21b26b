"""Reduced-precision rSVD against the FP64 oracle at the precision
configuration's shape: a planted-block graph with 100 blocks and average
degree 40, T = 10, d = 256, oversample 10, q = 3 (section 4.2, Algorithms
"Fast Randomized SVD" and "eigSVD"; the paper runs FP32 throughout).  The
dense steps run in FP32, or in BF16 on MFMA with FP32 accumulation, with the
Cholesky factorisations and eigen-solves in FP64.

The graph has 10^4 vertices (blocks of 100) so that the oracle's sparsifier
and FP64 randomized SVD finish in seconds, M = 5 T m, and 95% of the edges
inside blocks: the 100 planted directions then stand apart from the bulk of
the spectrum, and the relative gap g = (s_d' - s_d'+1) / s_1 at d' = 100
(about 0.35) is wide enough for a BF16 bound below pi/2.

Bars (u = 2^-24 for FP32, 2^-8 for BF16; k' = d + oversample): every stored
n x k' block carries a relative rounding error of at most u per entry, so
the products the randomized SVD factorises are perturbed by at most
sqrt(k') u s_1 in the 2-norm, and a few such roundings enter per power step:
  angle between the top-d' singular subspaces      <= 4 sqrt(k') u / g
  relative error of s_i, i <= d' (Weyl)             <= 4 sqrt(k') u s_1 / s_i
  Procrustes error of X0 = U S^(1/2) on the top d'  <= 4 sqrt(k') u / g
FP32 also checks every s_i, i <= d.  The test asserts that each bar is
below its trivial value (pi/2 for the angle, 1 for the relative errors), so
it can fail."""
import math

import numpy as np
import pytest

import oracle
from synth import workload
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu


def principal_angle(A, B):
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    r = qb - qa @ (qa.T @ qb)
    return float(np.arcsin(min(1.0, np.linalg.norm(r, 2))))


def procrustes_err(X, Xref):
    U, _, Vt = np.linalg.svd(X.T @ Xref)
    return float(np.linalg.norm(X @ (U @ Vt) - Xref) / np.linalg.norm(Xref))


@pytest.fixture(scope="module")
def c4_small():
    blocks, size, deg, intra = 100, 100, 40, 0.95
    g, p = workload("precision", sizes=[size] * blocks, p_in=intra * deg / (size - 1),
                    p_out=(1 - intra) * deg / (size * (blocks - 1)))
    p = dict(p, M=5 * p["T"] * g.m)
    assert (p["d"], p["oversample"], p["q"], p["T"]) == (256, 10, 3, 10)
    kp = p["d"] + p["oversample"]
    Mx = oracle.netmf_sparse(g, p)
    omega = oracle.gaussian_omega(g.n, kp, p["seed"])
    # all k' singular values of the last power step (to locate the gap)
    Uo, So, Vo = oracle.fast_rsvd(Mx, kp, 0, p["q"], omega)
    gaps = (So[:-1] - So[1:]) / So[0]
    dp = 2 + int(np.argmax(gaps[1:p["d"]]))          # widest gap past the first
    print(f"n={g.n} m={g.m} nnz={Mx.nnz} d'={dp} gap={gaps[dp - 1]:.4f}", flush=True)
    return g, p, Uo, So, dp, float(gaps[dp - 1])


@pytest.mark.parametrize("prec,u", [("f32", 2.0 ** -24), ("bf16", 2.0 ** -8)])
def test_reduced_precision_rsvd_against_oracle(lne, ctx, c4_small, prec, u):
    g, p, Uo, So, dp, gap = c4_small
    d, kp = p["d"], p["d"] + p["oversample"]
    assert dp == 100, "the planted directions must stand apart"
    pp = dict(p, precision=prec)
    rp, col = to_dev(g)
    counts, _ = lne.sparsify(ctx, rp, col, pp)
    M = lne.trunc_log(ctx, rp, col, pp, counts)
    counts.free()
    U, S, V, X0 = (x.double().cpu().numpy() for x in lne.rsvd(ctx, M, pp))
    M.free()
    base = 4 * math.sqrt(kp) * u
    angle_bar = base / gap
    sig_bar = base * So[0] / So[:dp]
    assert angle_bar < math.pi / 2 and np.all(sig_bar < 1), (angle_bar, sig_bar.max())
    angle = principal_angle(U[:, :dp], Uo[:, :dp])
    sig = np.abs(S[:dp] - So[:dp]) / So[:dp]
    X0o = Uo[:, :d] * np.sqrt(So[:d])
    pe = procrustes_err(X0[:, :dp], X0o[:, :dp])
    print(f"{prec}: angle {angle:.3e} (bar {angle_bar:.3e}), sigma {sig.max():.3e} "
          f"(bar {sig_bar.min():.3e}..{sig_bar.max():.3e}), X0 procrustes {pe:.3e}", flush=True)
    assert angle <= angle_bar
    assert np.all(sig <= sig_bar)
    assert pe <= angle_bar
    if prec == "f32":
        sig_all = np.abs(S - So[:d]) / So[:d]
        assert np.all(sig_all <= base * So[0] / So[:d])
