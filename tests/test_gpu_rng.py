"""Device Philox and Gaussian test matrix vs the oracle."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


def test_philox_counter_sweep(lne, ctx):
    import torch
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, size=(100_000, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [1, 0, 0, 0], [0, 0, 0, 0xFF000000]]
    for seed in (0, 0x299F31D0A4093822, 2 ** 64 - 1):
        d = torch.from_numpy(ctr.view(np.int32)).cuda()
        out = lne.philox(ctx, seed, d).cpu().numpy().view(np.uint32)
        np.testing.assert_array_equal(out, oracle.philox(seed, ctr))


@pytest.mark.parametrize("k", [1, 7, 42, 138])
def test_gaussian_matches_oracle(lne, ctx, k):
    import torch
    n = 3001
    ref = oracle.gaussian_omega(n, k, seed=11)
    g64 = lne.gaussian(ctx, n, k, 11, torch.float64).cpu().numpy()
    np.testing.assert_allclose(g64, ref, rtol=1e-13, atol=1e-13)
    g32 = lne.gaussian(ctx, n, k, 11, torch.float32, ld=(k + 7) // 8 * 8).cpu().numpy()
    np.testing.assert_allclose(g32, ref.astype(np.float32), rtol=2e-7, atol=1e-7)
    gbf = lne.gaussian(ctx, n, k, 11, torch.bfloat16, ld=(k + 7) // 8 * 8).float().cpu().numpy()
    np.testing.assert_allclose(gbf, ref, rtol=8e-3, atol=1e-2)
