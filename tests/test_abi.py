"""CPU checks of the C ABI: the library loads, exports every function that
include/lne.h declares, and rejects bad arguments on the host before any
GPU work (these calls never reach the HIP runtime)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
from tests import graphs_small as gs

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lne.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:lne_status|void|const char\s*\*|int64_t)\s*(lne_\w+)\s*\(",
                                 text, re.M)))


def test_every_declared_symbol_is_exported(lne):
    L = lne.load()
    names = declared()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    bound = {n for n, _, _ in lne.SIGNATURES}
    assert bound == set(names)


def test_version(lne):
    assert "gfx950" in lne.version()


def _ctx(lne):
    L = lne.load()
    h = ctypes.c_void_p()
    null_a = ctypes.cast(None, lne._ALLOC_T)
    null_f = ctypes.cast(None, lne._FREE_T)
    assert L.lne_ctx_create(ctypes.byref(h), None, null_a, null_f, None) == 0
    return L, h


def test_ctx_create_rejects_half_allocator(lne):
    L = lne.load()
    h = ctypes.c_void_p()
    a = lne._ALLOC_T(lambda n, u: None)
    null_f = ctypes.cast(None, lne._FREE_T)
    assert L.lne_ctx_create(ctypes.byref(h), None, a, null_f, None) == -1
    assert L.lne_ctx_create(None, None, ctypes.cast(None, lne._ALLOC_T), null_f, None) == -1


def _graph(n=10, n_arcs=20):
    g = __import__("paper_2302_07084_amd").Graph()
    g.n, g.n_arcs, g.row_ptr, g.col = n, n_arcs, 0x1000, 0x2000
    return g


@pytest.mark.parametrize("entry", ["lne_sparsify", "lne_sparsify_log"])
@pytest.mark.parametrize("field,value", [("T", 0), ("T", 17), ("b", 0), ("M", 1 << 40),
                                         ("precision", 7)])
def test_sparsify_rejects_bad_params(lne, entry, field, value):
    if entry == "lne_sparsify" and field == "precision":
        pytest.skip("the count matrix has no precision")
    L, h = _ctx(lne)
    p = lne.make_params(gs.params(T=3, m=10))
    setattr(p, field, value)
    out = lne.CsrStruct()
    rc = getattr(L, entry)(h, ctypes.byref(_graph()), ctypes.byref(p), ctypes.byref(out), None)
    assert rc == -1
    assert L.lne_last_error(h)
    L.lne_ctx_destroy(h)


def test_sparsify_rejects_bad_s(lne):
    L, h = _ctx(lne)
    for s in ([0.0, 0.0, 0.0], [0.5, -0.1, 0.6], [math.nan, 1, 1]):
        p = lne.make_params(gs.params(T=3, s=s, m=10))
        rc = L.lne_sparsify(h, ctypes.byref(_graph()), ctypes.byref(p), ctypes.byref(lne.CsrStruct()), None)
        assert rc == -1
    L.lne_ctx_destroy(h)


@pytest.mark.parametrize("n,n_arcs", [(0, 0), (5, 3), (5, -2), (5, 1 << 32), (1 << 31, 4)])
def test_graph_validation(lne, n, n_arcs):
    L, h = _ctx(lne)
    p = lne.make_params(gs.params(T=2, m=10))
    rc = L.lne_sparsify(h, ctypes.byref(_graph(n, n_arcs)), ctypes.byref(p),
                        ctypes.byref(lne.CsrStruct()), None)
    assert rc == -1
    L.lne_ctx_destroy(h)


@pytest.mark.parametrize("bits,n_arcs", [(16, 20), (-1, 20), (128, 20), (32, 1 << 31)])
def test_graph_index_bits_validation(lne, bits, n_arcs):
    # offsets are 64-bit (0 reads as 64) or 32-bit; 32-bit offsets cannot
    # address 2^31 arcs.  Rejected on the host, before any GPU work.
    L, h = _ctx(lne)
    p = lne.make_params(gs.params(T=2, m=10))
    g = _graph(10, n_arcs)
    g.index_bits = bits
    for entry in ("lne_sparsify", "lne_sparsify_log", "lne_embed"):
        out = lne.CsrStruct() if entry != "lne_embed" else ctypes.c_void_p(0x3000)
        arg = ctypes.byref(out) if entry != "lne_embed" else out
        rc = getattr(L, entry)(h, ctypes.byref(g), ctypes.byref(p), arg, None)
        assert rc == -1, entry
        assert b"index_bits" in L.lne_last_error(h) or b"32-bit" in L.lne_last_error(h)
    L.lne_ctx_destroy(h)


def test_linalg_param_validation(lne):
    L, h = _ctx(lne)
    base = gs.params(T=2, m=10, d=4, oversample=2, q=1)
    for bad in (dict(q=0), dict(d=0), dict(d=300), dict(d=8, oversample=4), dict(cheb_k=-1),
                dict(theta=-1.0), dict(precision=7)):
        p = lne.make_params(dict(base, **bad))
        rc = L.lne_embed(h, ctypes.byref(_graph()), ctypes.byref(p), ctypes.c_void_p(0x3000), None)
        assert rc in (-1, -5), bad
    L.lne_ctx_destroy(h)


def test_sampler_plan_matches_oracle(lne):
    rng = np.random.default_rng(0)
    for T in (1, 3, 10, 16):
        for _ in range(5):
            s = rng.dirichlet(np.ones(T))
            s[rng.random(T) < 0.2] = 0.0
            if s.sum() == 0:
                s[0] = 1.0
            m = int(rng.integers(1, 10 ** 7))
            M = int(rng.integers(1, 10 ** 10))
            p = dict(T=T, s=s, M=M, b=1, C=1.0, seed=0)
            assert lne.sampler_plan(p, 2 * m)[0:2] == oracle.plan(T, s, M, m)[0:2]
            np.testing.assert_array_equal(lne.sampler_plan(p, 2 * m)[2], oracle.plan(T, s, M, m)[2])
            assert lne.slots_per_edge(p, 2 * m) == M // m + (1 if M % m else 0)


def test_link_rank_rejects_bad_arguments(lne):
    L, h = _ctx(lne)
    X, P, N, Mx = (ctypes.c_void_p(a) for a in (0x10000, 0x20000, 0x30000, 0x40000))
    F32, F64 = lne.F32, lne.F64
    good = dict(X=X, n=100, d=32, ldx=32, dt=F32, pos=P, h=10, neg=N, K=5, hk=10)
    for bad in (dict(X=None), dict(n=0), dict(d=0), dict(d=4096, ldx=4096), dict(ldx=16),
                dict(h=0), dict(K=0), dict(hk=0), dict(dt=lne.BF16), dict(pos=None),
                dict(neg=None), dict(X=ctypes.c_void_p(0x10008)), dict(ldx=34)):
        a = dict(good, **bad)
        rc = L.lne_link_rank(h, a["X"], a["n"], a["d"], a["ldx"], a["dt"], a["pos"], a["h"],
                             a["neg"], a["K"], a["hk"], None, None, Mx)
        assert rc == -1, bad
    L.lne_ctx_destroy(h)


def test_sparse_omega_rejects_bad_arguments(lne):
    L, h = _ctx(lne)
    out = ctypes.c_void_p(0x10000)
    for n, k, o in ((-1, 8, out), (10, 0, out), (10, 1025, out), (10, 8, None),
                    (10, 8, ctypes.c_void_p(0x10002))):
        assert L.lne_sparse_omega(h, n, k, 1, o) == -1, (n, k)
    A = lne.CsrStruct()
    A.n_rows, A.n_cols, A.nnz, A.val_type = 4, 4, 0, lne.F32
    assert L.lne_spmm_sparse_omega(h, ctypes.byref(A), ctypes.c_void_p(0x10004),
                                   ctypes.c_void_p(0x20000), 8, 8, lne.F32) == -1
    assert L.lne_spmm_sparse_omega(h, ctypes.byref(A), ctypes.c_void_p(0x10000),
                                   ctypes.c_void_p(0x20000), 8, 2000, lne.F32) == -1
    L.lne_ctx_destroy(h)


def test_batched_trials_reject_weighted_graphs(lne):
    L, h = _ctx(lne)
    g = _graph()
    g.weight = 0x5000
    p = lne.make_params(gs.params(T=3, m=10))
    rc = L.lne_sparsify_channels(h, ctypes.byref(g), ctypes.byref(p), ctypes.byref(lne.CsrStruct()),
                                 None)
    assert rc == -5
    assert b"unweighted" in L.lne_last_error(h)
    L.lne_ctx_destroy(h)


def test_graph_spmm_rejects_bad_arguments(lne):
    """Checked on the host before the device graph check runs."""
    L, h = _ctx(lne)
    Z, O = ctypes.c_void_p(0x10000), ctypes.c_void_p(0x20000)
    good = dict(Z=Z, ld=8, k=8, dt=lne.F32, out=O)
    for bad in (dict(Z=None), dict(out=None), dict(k=0), dict(ld=4), dict(dt=lne.BF16),
                dict(dt=lne.U64), dict(out=Z)):
        a = dict(good, **bad)
        rc = L.lne_graph_spmm(h, ctypes.byref(_graph()), a["Z"], a["ld"], a["k"], a["dt"],
                              ctypes.c_double(1.0), ctypes.c_double(-1.0), a["out"])
        assert rc == -1, bad
    rc = L.lne_graph_spmm(h, ctypes.byref(_graph(0, 0)), Z, 8, 8, lne.F32, ctypes.c_double(1.0),
                          ctypes.c_double(-1.0), O)
    assert rc == -1
    L.lne_ctx_destroy(h)
