"""lne_graph_stats (the search's graph descriptors) against the oracle's
graph_stats on the same graphs: degree moments, median and Hill exponent to
rounding, the closed-wedge count exactly (the same Philox draws on both
sides), and the spectral gap of the same subspace iteration to 1e-9."""
import math

import numpy as np
import pytest

from oracle import graphstats as gst
from synth import graphs as sg
from tests import graphs_small as gs
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu

GRAPHS = {
    "complete12": lambda: gs.complete(12),
    "cycle12": lambda: gs.cycle(12),
    "path30": lambda: gs.path(30),
    "star50": lambda: gs.star(50),
    "sbm2000": lambda: sg.sbm([100] * 20, 0.2, 0.01, seed=3),
    "chunglu4000": lambda: sg.chung_lu(4000, 40000, 2.1, seed=2),   # isolated vertices too
}


@pytest.mark.parametrize("name", list(GRAPHS))
def test_graph_stats_match_oracle(lne, ctx, name):
    g = GRAPHS[name]()
    W, iters, seed = 3000, 200, 7
    rp, col = to_dev(g)
    got = lne.graph_stats(ctx, rp, col, seed=seed, wedges=W, iters=iters)
    ref = gst.graph_stats(g, seed=seed, wedges=W, iters=iters)
    print(name, "gpu", got, "oracle", ref, flush=True)
    np.testing.assert_allclose(got[:6], ref[:6], rtol=1e-12, atol=1e-14)
    assert round(got[6] * W) == gst.wedge_closed(g, seed, W)
    assert abs(got[7] - ref[7]) <= 1e-9


def test_graph_stats_rejects_bad_input(lne, ctx):
    import torch
    g = gs.cycle(8)
    rp, col = to_dev(g)
    with pytest.raises(lne.LneError):
        lne.graph_stats(ctx, rp, col, wedges=0)
    with pytest.raises(lne.LneError):
        lne.graph_stats(ctx, rp, col, iters=0)
    empty_rp = torch.zeros(5, dtype=torch.int64, device="cuda")
    empty_col = torch.zeros(0, dtype=torch.int32, device="cuda")
    with pytest.raises(lne.LneError):
        lne.graph_stats(ctx, empty_rp, empty_col)
