"""The headline FP32 path end to end against the FP64 oracle on the mid
power-law workload (Chung-Lu, 10^4 vertices, 3.3 10^5 edges, T = 10,
s ~ Dirichlet(1), d = 128, q = 1, k = 10, theta = 0.5, mu = 0.2) with
M = 20 T m instead of 2000 T m so that the oracle finishes in seconds.

* The randomized SVD of the matrix lne_embed factorises (lne_sparsify_log, the
  aggregation with Eq. (1) fused) against oracle.fast_rsvd of the oracle's own
  matrix: the principal angle of the top d' singular vectors (d' the largest
  index <= d with a relative gap of at least 1e-3) within 100 sqrt(k') u / gap
  and the singular values within 10 sqrt(k') u s_1 / s_i (the tolerances of
  the method's parity contract), and X0 within its derived Procrustes bar.
* The embedding lne_embed returns against oracle.embed: Procrustes error
  within the bar derived in tests/bars.py (randomized SVD perturbation,
  propagation norm and rounding, final scaling).
"""
import math

import numpy as np
import pytest

import oracle
from synth import workload
from tests import bars
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def principal_angle(A, B):
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    r = qb - qa @ (qa.T @ qb)
    return float(np.arcsin(min(1.0, np.linalg.norm(r, 2))))


def procrustes_err(X, Xref):
    U, _, Vt = np.linalg.svd(X.T @ Xref)
    return float(np.linalg.norm(X @ (U @ Vt) - Xref) / np.linalg.norm(Xref))


@pytest.fixture(scope="module")
def mid():
    g, p = workload("mid")
    p = dict(p, M=20 * p["T"] * g.m)
    assert p["precision"] == "f32"
    ref = oracle.embed(g, p, return_stages=True)
    kp = p["d"] + p["oversample"]
    _, S_all, _ = oracle.fast_rsvd(ref["M"], kp, 0, p["q"], ref["omega"])
    print(f"mid: n={g.n} m={g.m} nnz={ref['M'].nnz}", flush=True)
    return g, p, ref, S_all


def test_fp32_rsvd_of_the_embedding_matrix(lne, ctx, mid):
    g, p, ref, S_all = mid
    d, kp = p["d"], p["d"] + p["oversample"]
    rp, col = to_dev(g)
    M, _ = lne.sparsify_log(ctx, rp, col, p)
    U, S, V, X0 = (x.double().cpu().numpy() for x in lne.rsvd(ctx, M, p))
    M.free()
    gaps = (S_all[:-1] - S_all[1:]) / S_all[0]
    dp = max(i + 1 for i in range(d) if gaps[i] >= 1e-3)
    angle = principal_angle(U[:, :dp], ref["U"][:, :dp])
    angle_bar = 100 * math.sqrt(kp) * U32 / gaps[dp - 1]
    sig = np.abs(S - ref["S"]) / ref["S"]
    sig_bar = 10 * math.sqrt(kp) * U32 * ref["S"][0] / ref["S"]
    pe = procrustes_err(X0, ref["X0"])
    pe_bar = bars.x0_bar(S_all, d, kp, U32)
    print(f"d'={dp} angle {angle:.3e} (bar {angle_bar:.3e}); sigma {sig.max():.3e}; "
          f"X0 procrustes {pe:.3e} (bar {pe_bar:.3e})", flush=True)
    assert angle <= angle_bar < math.pi / 2
    assert np.all(sig <= sig_bar)
    assert pe <= pe_bar < 0.5


def test_fp32_embedding_against_oracle(lne, ctx, mid):
    g, p, ref, S_all = mid
    d, kp = p["d"], p["d"] + p["oversample"]
    rp, col = to_dev(g)
    X, st = lne.embed(ctx, rp, col, p)
    X = X.double().cpu().numpy()
    assert st["nnz_log"] == ref["M"].nnz
    trial = dict(k=p["cheb_k"], theta=p["theta"], mu=p["mu"])
    bar = bars.embedding_bar(g, ref["X0"], ref["Xsp"], S_all, d, kp, trial)
    err = procrustes_err(X, ref["X"])
    print(f"embedding procrustes {err:.3e} (bar {bar:.3e})", flush=True)
    assert bar < 0.5
    assert err <= bar
