"""FP32 and BF16-MFMA paths against the FP64 path on the mid power-law
workload (the FP64 path itself is pinned to the oracle on the tiny workload)."""
import math

import numpy as np
import pytest

from synth import workload
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu


def principal_angle(A, B):
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    r = qb - qa @ (qa.T @ qb)
    return float(np.arcsin(min(1.0, np.linalg.norm(r, 2))))


def test_reduced_precision_rsvd_within_bar(lne, ctx):
    g, p = workload("mid")
    p = dict(p, M=200 * p["T"] * g.m)
    rp, col = to_dev(g)
    out = {}
    for prec in ("f64", "f32", "bf16"):
        pp = dict(p, precision=prec)
        counts, _ = lne.sparsify(ctx, rp, col, pp)
        M = lne.trunc_log(ctx, rp, col, pp, counts)
        U, S, V, X0 = lne.rsvd(ctx, M, pp)
        out[prec] = (U.double().cpu().numpy(), S.cpu().numpy())
    U64, S64 = out["f64"]
    gaps = (S64[:-1] - S64[1:]) / S64[0]
    dp = max(i + 1 for i in range(len(gaps)) if gaps[i] >= 1e-3)
    kp = p["d"] + p["oversample"]
    for prec, u in (("f32", 2.0 ** -24), ("bf16", 2.0 ** -8)):
        U, S = out[prec]
        bar = 100 * math.sqrt(kp) * u / gaps[dp - 1]
        angle = principal_angle(U[:, :dp], U64[:, :dp])
        assert angle <= bar, (prec, angle, bar, dp)
        assert np.max(np.abs(S[:dp] - S64[:dp]) / S64[:dp]) <= 10 * math.sqrt(kp) * u * S64[0] / S64[dp - 1]
