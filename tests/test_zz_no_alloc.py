"""The allocation-free eigSVD entry point (lne_eigsvd_noalloc) against
lne_eigsvd, called through the C ABI on a context whose allocator records
every request and refuses it: three calls in a row on one device (the
library's fixed array keeps the previous call's contents), the later ones
with smaller inputs.

* FP64, n = 2 10^5, k = 266: the array holds fewer per-workgroup partial
  Grams than lne_eigsvd uses, so the Gram is summed in another order: the
  singular values within 10 sqrt(k) u (s_1 / s_i)^2 (an eigenvalue of the
  Gram moves by a few u s_1^2), Y's reconstruction U S V^T and the Gram
  V S^2 V^T within 1e-11 of lne_eigsvd's.
* FP32, n = 5000, k = 40 and BF16, n = 3000, k = 138: the same number of
  workgroups as lne_eigsvd, so the results are bit-identical.
"""
import ctypes
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53


def _rand_y(n, k, seed, cond):
    rng = np.random.default_rng(seed)
    Q1, _ = np.linalg.qr(rng.standard_normal((n, k)))
    Q2, _ = np.linalg.qr(rng.standard_normal((k, k)))
    return (Q1 * np.logspace(0, -math.log10(cond), k)) @ Q2


def _counting_ctx(lne):
    """A raw context on the default stream whose allocator counts requests and
    returns NULL (any allocation would make the call fail with ENOMEM)."""
    L = lne.load()
    calls = []

    def alloc(size, user):
        calls.append(size)
        return None

    def free(ptr, user):
        calls.append(-1)

    fa, ff = lne._ALLOC_T(alloc), lne._FREE_T(free)
    h = ctypes.c_void_p()
    assert L.lne_ctx_create(ctypes.byref(h), None, fa, ff, None) == 0
    return L, h, calls, (fa, ff)


def _noalloc(L, h, Y):
    import torch
    n, k = Y.shape
    ut = torch.float32 if Y.dtype == torch.bfloat16 else Y.dtype
    U = torch.empty((n, k), dtype=ut, device=Y.device)
    S = torch.empty(k, dtype=torch.float64, device=Y.device)
    V = torch.empty((k, k), dtype=torch.float64, device=Y.device)
    torch.cuda.synchronize()
    code = {torch.float64: 0, torch.float32: 1, torch.bfloat16: 2}[Y.dtype]
    rc = L.lne_eigsvd_noalloc(h, Y.data_ptr(), n, k, Y.stride(0), code, U.data_ptr(),
                              U.stride(0), S.data_ptr(), V.data_ptr())
    assert rc == 0, L.lne_last_error(h)
    torch.cuda.synchronize()
    return U, S, V


def test_eigsvd_noalloc_matches_eigsvd(lne, ctx):
    import torch
    L, h, calls, keep = _counting_ctx(lne)
    # 1: FP64, wide k, fewer Gram workgroups than lne_eigsvd
    n, k = 200_000, 266
    Y = torch.from_numpy(_rand_y(n, k, seed=1, cond=1e3)).cuda()
    U0, S0, V0 = (x.cpu().numpy() for x in lne.eigsvd(ctx, Y))
    U1, S1, V1 = (x.cpu().numpy() for x in _noalloc(L, h, Y))
    assert calls == []
    np.testing.assert_array_less(np.abs(S1 - S0) / S0, 10 * math.sqrt(k) * U64 * (S0[0] / S0) ** 2)
    Yh = Y.cpu().numpy()
    for U_, S_, V_ in ((U0, S0, V0), (U1, S1, V1)):
        assert np.linalg.norm((U_ * S_) @ V_.T - Yh) <= 1e-11 * np.linalg.norm(Yh)
    G0, G1 = (V0 * S0 ** 2) @ V0.T, (V1 * S1 ** 2) @ V1.T
    assert np.linalg.norm(G1 - G0) <= 1e-11 * np.linalg.norm(G0)
    # 2: FP32, smaller: same launch shapes, identical bits
    Y2 = torch.from_numpy(_rand_y(5000, 40, seed=2, cond=1e2)).float().cuda()
    ref = [x.cpu().numpy() for x in lne.eigsvd(ctx, Y2)]
    got = [x.cpu().numpy() for x in _noalloc(L, h, Y2)]
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a, b)
    # 3: BF16 rows with a padded leading dimension, smaller again
    k3 = 138
    Y3 = torch.zeros((3000, 144), dtype=torch.bfloat16, device="cuda")
    Y3[:, :k3] = torch.from_numpy(_rand_y(3000, k3, seed=3, cond=10.0)).to(torch.bfloat16)
    ref = [x.cpu().numpy() for x in lne.eigsvd(ctx, Y3[:, :k3])]
    got = [x.cpu().numpy() for x in _noalloc(L, h, Y3[:, :k3])]
    for a, b in zip(got, ref):
        np.testing.assert_array_equal(a, b)
    assert calls == []
    L.lne_ctx_destroy(h)
    del keep


def test_eigsvd_noalloc_rejects_bad_arguments(lne):
    L, h, calls, keep = _counting_ctx(lne)
    Y, U, S, V = (ctypes.c_void_p(a) for a in (0x10000, 0x20000, 0x30000, 0x40000))
    for args in ((None, 10, 4, 4, 0), (Y, 0, 4, 4, 0), (Y, 10, 0, 4, 0), (Y, 10, 4, 3, 0),
                 (Y, 10, 4, 4, 7), (Y, 400, 289, 289, 0)):
        y, n, k, ld, dt = args
        rc = L.lne_eigsvd_noalloc(h, y, n, k, ld, dt, U, k, S, V)
        assert rc in (-1, -5), args
    assert calls == []
    L.lne_ctx_destroy(h)
    del keep
