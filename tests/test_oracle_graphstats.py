"""Pins of the oracle's graph descriptors (oracle/graphstats.py, reading R22)
against closed forms and brute force: graphs whose degree sequence, triangle
count and normalized-adjacency spectrum are known exactly."""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as sla

from oracle import graphstats as gst
from synth import graphs as sg
from tests import graphs_small as gs


def test_complete_graph():
    # K_n: every degree n-1, every wedge closes; N = (J - I)/(n-1) has
    # lambda_2 = -1/(n-1); the median is n-1, so the Hill tail is all of it
    n = 12
    st = gst.graph_stats(gs.complete(n), seed=3, wedges=500, iters=50)
    assert st[0] == pytest.approx(math.log(n), abs=1e-14)
    assert st[1] == pytest.approx(math.log(n * (n - 1) / 2), abs=1e-14)
    assert st[2] == pytest.approx(math.log(n - 1), abs=1e-14)
    assert st[3] == 0.0
    assert st[4] == pytest.approx(math.log(n - 1), abs=1e-14)
    assert st[5] == pytest.approx(1 + 1 / math.log((n - 1) / (n - 1.5)), rel=1e-13)
    assert st[6] == 1.0
    assert st[7] == pytest.approx(1 + 1 / (n - 1), abs=1e-12)


def test_cycle_and_path():
    # C_n: no triangles, lambda_2 = cos(2 pi / n).  P_n: degrees (1, 2, ..., 2,
    # 1), median 2, tail = the n-2 inner vertices, lambda_2 = cos(pi / (n-1))
    n = 12
    st = gst.graph_stats(gs.cycle(n), seed=3, wedges=500, iters=50)
    assert st[3] == 0.0 and st[6] == 0.0
    assert st[7] == pytest.approx(1 - math.cos(2 * math.pi / n), abs=1e-12)
    n = 30
    st = gst.graph_stats(gs.path(n), seed=3, wedges=500, iters=200)
    d = np.array([1] + [2] * (n - 2) + [1], float)
    assert st[3] == pytest.approx(d.std() / d.mean(), rel=1e-13)
    assert st[5] == pytest.approx(1 + 1 / math.log(2 / 1.5), rel=1e-13)
    assert st[6] == 0.0
    assert st[7] == pytest.approx(1 - math.cos(math.pi / (n - 1)), abs=1e-10)


def test_star():
    # S_n (hub + n-1 leaves): median degree 1, so x_min = 1 and every vertex
    # is in the tail; the only wedges are leaf pairs, never adjacent; the
    # spectrum of N is {1, 0 (n-2 times), -1}
    n = 50
    st = gst.graph_stats(gs.star(n), seed=3, wedges=500, iters=20)
    assert st[4] == pytest.approx(math.log(n - 1), abs=1e-14)
    assert st[5] == pytest.approx(1 + n / ((n - 1) * math.log(2) + math.log((n - 1) / 0.5)),
                                  rel=1e-13)
    assert st[6] == 0.0
    assert st[7] == pytest.approx(1.0, abs=1e-12)


def test_wedge_estimator_matches_brute_force_mean_local_clustering():
    # a wedge with a uniform centre (degree >= 2) and a uniform pair of its
    # neighbours closes with probability mean_v t_v / C(d_v, 2); brute force
    # counts the triangles t_v of every vertex
    g = sg.sbm([60] * 5, 0.3, 0.02, seed=4)
    A = sp.csr_matrix((np.ones(len(g.col)), g.col, g.rowptr), shape=(g.n, g.n))
    tri = np.asarray((A @ A).multiply(A).sum(axis=1)).ravel() / 2
    d = np.diff(g.rowptr)
    ok = d >= 2
    cbar = float(np.mean(tri[ok] / (d[ok] * (d[ok] - 1) / 2)))
    W = 20000
    est = gst.wedge_closed(g, seed=11, wedges=W) / W
    sd = math.sqrt(cbar * (1 - cbar) / W)
    assert abs(est - cbar) <= 4 * sd
    assert gst.wedge_closed(g, seed=11, wedges=W) == gst.wedge_closed(g, seed=11, wedges=W)


def test_subspace_iteration_reaches_the_exact_lambda2():
    # a power-law graph, where lambda_2 is separated from the rest: the
    # 200-step estimate equals Lanczos to 1e-6; on a planted-partition graph,
    # whose lambda_2 sits at the edge of a dense bulk, the estimate
    # approaches it from below and is within 5e-3
    for g, tol in [(sg.chung_lu(4000, 40000, 2.1, seed=2), 1e-6),
                   (sg.sbm([100] * 20, 0.2, 0.01, seed=3), 5e-3)]:
        d = np.diff(g.rowptr).astype(float)
        s = np.where(d > 0, 1 / np.sqrt(np.where(d > 0, d, 1)), 0)
        A = sp.csr_matrix((np.ones(len(g.col)), g.col, g.rowptr), shape=(g.n, g.n))
        N = sp.diags(s) @ A @ sp.diags(s)
        lam = np.sort(sla.eigsh(N, k=2, which="LA", return_eigenvectors=False, tol=1e-13))
        est = gst.spectral_lambda2(g, seed=5, iters=200)
        assert est <= lam[0] + 1e-10
        assert lam[0] - est <= tol
