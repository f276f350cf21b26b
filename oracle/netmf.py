"""ORACLE -- test infrastructure, not part of the product.

FP64 reference of every step of the sparsified-NetMF hot path.  Each function
names the passage of arXiv 2302.07084 it follows.  Sampling, aggregation and
the truncated logarithm are in ``sampler.c`` (plain C, called through
ctypes); the linear algebra uses numpy/scipy library routines as its steps
(matrix products, LAPACK symmetric eigensolver) with no blocking or fusion.

Readings of points the paper leaves open are stated where they are used; the
full list is in the design notes of the repository.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import scipy.sparse as sp
import scipy.special

from . import build as _build

F_BITS = 16                 # fixed-point fraction bits of sample weights
FLAG_VANILLA_RSVD = 2       # params["flags"] bit: the vanilla randomized SVD
FLAG_SPARSE_OMEGA = 4       # params["flags"] bit: sparse-sign test matrix
TAG_SPARSE_OMEGA = 5 << 24  # Philox counter tag of the sparse-sign test matrix
SPARSE_OMEGA_NNZ = 8        # signed entries per row
TAG_OMEGA = 3 << 24         # Philox counter tag of the Gaussian test matrix

_LIB = None


def lib():
    """ctypes handle of liboracle.so (built on first use if absent)."""
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i64, u64, i32, f64 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
        L.ora_philox.argtypes = [u64, P, i64, P]
        L.ora_plan.argtypes = [i32, P, u64, i64, P, P, P]
        L.ora_sample_slots.argtypes = [i64, P, P, P, i32, P, u64, f64, i32, u64, i64, i64, i64,
                                       P, P, P, P, P, P, P]
        L.ora_sample_slots.restype = i64
        L.ora_count_rows.argtypes = [i64, P, P, P, i32, P, u64, f64, i32, u64, i64, i64, i64,
                                     i64, i32, i32, P, P, P, P, P, P]
        L.ora_count_rows.restype = i32
        L.ora_count_rows_list.argtypes = [i64, P, P, P, i32, P, u64, f64, i32, u64, i64, i64, P,
                                          i64, i32, P, P, P, P, P, P]
        L.ora_count_rows_list.restype = i32
        L.ora_free.argtypes = [P]
        L.ora_trunc_log.argtypes = [i64, i64, P, P, P, P, u64, u64, u64, u64, P, P]
        _LIB = L
    return _LIB


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _graph_arrays(g):
    return (np.ascontiguousarray(g.rowptr, dtype=np.int64),
            np.ascontiguousarray(g.col, dtype=np.int32))


def _weights(g):
    """Arc weights as a C pointer argument (None: unweighted graph) and the
    array that keeps it alive."""
    w = getattr(g, "weight", None)
    if w is None:
        return None, None
    w = np.ascontiguousarray(w, dtype=np.uint32)
    return _p(w), w


def degrees(g) -> np.ndarray:
    """d_u = sum_v A_uv (int64): the arc count on an unweighted graph."""
    w = getattr(g, "weight", None)
    if w is None:
        return np.diff(np.asarray(g.rowptr, dtype=np.int64))
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    return np.bincount(rows, weights=np.asarray(w, np.float64), minlength=g.n).astype(np.int64)


def volume(g) -> int:
    """vol(G) = sum_u d_u."""
    return int(degrees(g).sum())


def _rc_check(rc):
    if rc == -1:
        raise MemoryError("oracle aggregation ran out of memory")
    if rc == -2:
        raise OverflowError("weight sum exceeds uint64")
    if rc == -3:
        raise ValueError("edge id out of range")
    if rc == -4:
        raise ValueError("zero weight or weighted degree >= 2^32")


def _s_array(params):
    s = np.ascontiguousarray(np.asarray(params["s"], dtype=np.float64))
    assert len(s) == params["T"]
    return s


def _coin_args(params):
    C = params.get("C")
    no_ds = 1 if (C is None or (isinstance(C, float) and math.isinf(C))) else 0
    return (0.0 if no_ds else float(C)), no_ds


# --------------------------------------------------------------------------
# Random numbers
# --------------------------------------------------------------------------
def philox(seed: int, ctr: np.ndarray) -> np.ndarray:
    """Philox4x32-10 blocks for counters ``ctr`` (N x 4 uint32), key = seed."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    out = np.empty_like(ctr)
    lib().ora_philox(ctypes.c_uint64(seed), _p(ctr), ctr.shape[0], _p(out))
    return out


def plan(T: int, s, M: int, m: int):
    """Integer constants of the sampler: floor(M/m), the Bernoulli threshold of
    frac(M/m) and the length thresholds of Multinomial(s) (Algorithm
    "Downsampled Per-Edge PathSampling", the n_e and r draws)."""
    s = np.ascontiguousarray(np.asarray(s, dtype=np.float64))
    base = np.zeros(1, np.uint64)
    thr = np.zeros(1, np.uint64)
    theta = np.zeros(T, np.uint64)
    lib().ora_plan(T, _p(s), M, m, _p(base), _p(thr), _p(theta))
    return int(base[0]), int(thr[0]), theta


# --------------------------------------------------------------------------
# Sparsifier (section 5.2)
# --------------------------------------------------------------------------
def sample_slots(g, params, e_begin: int = 0, e_end: int | None = None):
    """Every sample slot (e, j) of edges [e_begin, e_end): accepted flag, r,
    endpoints (u', v') and fixed-point weight (0 if rejected)."""
    rp, col = _graph_arrays(g)
    wp, _keep = _weights(g)
    m = g.m
    if e_end is None:
        e_end = m
    s = _s_array(params)
    C, no_ds = _coin_args(params)
    cap = 1 << 16
    while True:
        out = dict(e=np.empty(cap, np.int64), j=np.empty(cap, np.uint32),
                   acc=np.empty(cap, np.uint8), r=np.empty(cap, np.uint8),
                   a=np.empty(cap, np.int32), b=np.empty(cap, np.int32),
                   w=np.empty(cap, np.uint64))
        k = lib().ora_sample_slots(g.n, _p(rp), _p(col), wp, params["T"], _p(s),
                                   int(params["M"]), C, no_ds, int(params["seed"]),
                                   e_begin, e_end, cap, _p(out["e"]), _p(out["j"]),
                                   _p(out["acc"]), _p(out["r"]), _p(out["a"]),
                                   _p(out["b"]), _p(out["w"]))
        if k == -(1 << 63):
            _rc_check(-4)
        if k >= 0:
            return {key: v[:k] for key, v in out.items()}
        cap = -k


def count_csr(g, params, row_lo: int = 0, row_hi: int | None = None,
              nthreads: int | None = None, e_begin: int = 0, e_end: int = -1,
              channels: bool = False):
    """Aggregated count matrix W (fixed point, 2^-16 units) restricted to rows
    [row_lo, row_hi), from the samples of edges [e_begin, e_end) (all edges
    by default): returns (rowptr, col, W, attempted, accepted).  With
    ``channels`` the length r (drawn from s as always) is kept: column
    (b << 4) | (r - 1).  Equal
    pairs are summed exactly in uint64 (section 5.2, sparse parallel hashing;
    here a sort of the sample triples)."""
    rp, col = _graph_arrays(g)
    wp, _keep = _weights(g)
    if row_hi is None:
        row_hi = g.n
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    s = _s_array(params)
    C, no_ds = _coin_args(params)
    prp = ctypes.c_void_p()
    pcol = ctypes.c_void_p()
    pw = ctypes.c_void_p()
    nnz = ctypes.c_int64()
    att = ctypes.c_uint64()
    acc = ctypes.c_uint64()
    rc = lib().ora_count_rows(g.n, _p(rp), _p(col), wp, params["T"], _p(s), int(params["M"]),
                              C, no_ds, int(params["seed"]), row_lo, row_hi, e_begin, e_end,
                              1 if channels else 0, nthreads,
                              ctypes.byref(prp), ctypes.byref(pcol), ctypes.byref(pw),
                              ctypes.byref(nnz), ctypes.byref(att), ctypes.byref(acc))
    _rc_check(rc)
    rows = row_hi - row_lo
    k = nnz.value
    R = np.ctypeslib.as_array(ctypes.cast(prp, ctypes.POINTER(ctypes.c_int64)), (rows + 1,)).copy()
    Cc = (np.ctypeslib.as_array(ctypes.cast(pcol, ctypes.POINTER(ctypes.c_int32)), (k,)).copy()
          if k else np.zeros(0, np.int32))
    W = (np.ctypeslib.as_array(ctypes.cast(pw, ctypes.POINTER(ctypes.c_uint64)), (k,)).copy()
         if k else np.zeros(0, np.uint64))
    for ptr in (prp, pcol, pw):
        lib().ora_free(ptr)
    return R, Cc, W, att.value, acc.value


def edge_ids(g):
    """Edge id of every arc: the arcs (u, v) with u < v numbered in CSR order;
    arc (v, u) gets the id of its mirror.  Returns an int64 array of 2m."""
    rp, col = _graph_arrays(g)
    n = g.n
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    up = col > rows
    ids = np.full(len(col), -1, np.int64)
    ids[up] = np.arange(int(up.sum()), dtype=np.int64)
    # the mirror of arc (u, v), u > v, sits in row v at column u; the keys
    # row * n + col are ascending over the whole CSR
    lo = np.flatnonzero(~up)
    key = rows * n + col.astype(np.int64)
    pos = np.searchsorted(key, col[lo].astype(np.int64) * n + rows[lo])
    ids[lo] = ids[pos]
    return ids


def edge_ids_of(g, arcs):
    """Edge ids of the arcs at CSR positions `arcs` (see edge_ids), from one
    pass over the graph for the per-row counts of arcs (u, v) with u < v."""
    rp, col = _graph_arrays(g)
    n = g.n
    arcs = np.asarray(arcs, np.int64)
    rows_all = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    up = (col > rows_all).astype(np.int64)
    del rows_all
    cum = np.concatenate([[0], np.cumsum(up)])        # upper arcs before each position
    first_upper = rp[1:] - (cum[rp[1:]] - cum[rp[:-1]])
    upper_before = cum[rp[:-1]]
    a_row = np.searchsorted(rp, arcs, side="right") - 1
    a_col = col[arcs].astype(np.int64)
    out = np.empty(len(arcs), np.int64)
    fwd = a_col > a_row
    out[fwd] = upper_before[a_row[fwd]] + (arcs[fwd] - first_upper[a_row[fwd]])
    bwd = ~fwd
    # mirror (x, b) of arc (b, x), x < b: its position inside row x
    x, b = a_col[bwd], a_row[bwd]
    pos = np.array([rp[xx] + np.searchsorted(col[rp[xx]:rp[xx + 1]], bb)
                    for xx, bb in zip(x, b)], dtype=np.int64)
    out[bwd] = upper_before[x] + (pos - first_upper[x])
    return out


def count_csr_edges(g, params, row_lo: int, row_hi: int, edges, nthreads: int | None = None):
    """count_csr restricted to the samples of the listed edges (distinct edge
    ids): the rows [row_lo, row_hi) of the count matrix are exact whenever the
    list holds every edge whose samples can reach those rows."""
    rp, col = _graph_arrays(g)
    wp, _keep = _weights(g)
    if nthreads is None:
        nthreads = min(16, os.cpu_count() or 1)
    s = _s_array(params)
    C, no_ds = _coin_args(params)
    el = np.ascontiguousarray(np.unique(np.asarray(edges, np.int64)))
    prp, pcol, pw = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
    nnz, att, acc = ctypes.c_int64(), ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib().ora_count_rows_list(g.n, _p(rp), _p(col), wp, params["T"], _p(s), int(params["M"]),
                                   C, no_ds, int(params["seed"]), row_lo, row_hi, _p(el), len(el),
                                   nthreads, ctypes.byref(prp), ctypes.byref(pcol),
                                   ctypes.byref(pw), ctypes.byref(nnz), ctypes.byref(att),
                                   ctypes.byref(acc))
    _rc_check(rc)
    rows = row_hi - row_lo
    k = nnz.value
    R = np.ctypeslib.as_array(ctypes.cast(prp, ctypes.POINTER(ctypes.c_int64)), (rows + 1,)).copy()
    Cc = (np.ctypeslib.as_array(ctypes.cast(pcol, ctypes.POINTER(ctypes.c_int32)), (k,)).copy()
          if k else np.zeros(0, np.int32))
    W = (np.ctypeslib.as_array(ctypes.cast(pw, ctypes.POINTER(ctypes.c_uint64)), (k,)).copy()
         if k else np.zeros(0, np.uint64))
    for ptr in (prp, pcol, pw):
        lib().ora_free(ptr)
    return R, Cc, W


def trunc_log(g, params, rowptr, col, W, row_lo: int = 0):
    """Eq. (1): x = vol 2m/(2bM) * (W/2^F) / (d_a d_b) (vol = 2m unweighted:
    vol^2/(2bM)); keep x > 1 (exact integer test), value log x.  Returns
    (keep mask, values)."""
    deg = np.ascontiguousarray(degrees(g), dtype=np.int64)
    rows = len(rowptr) - 1
    keep = np.zeros(len(col), np.uint8)
    val = np.zeros(len(col), np.float64)
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    W = np.ascontiguousarray(W, dtype=np.uint64)
    lib().ora_trunc_log(rows, row_lo, _p(deg), _p(rowptr), _p(col), _p(W),
                        volume(g), g.n_arcs, int(params["b"]), int(params["M"]), _p(keep),
                        _p(val))
    return keep.astype(bool), val


def compact(rowptr, col, keep, val):
    """Drop the entries trunc_log removed; returns (rowptr, col, val)."""
    rows = len(rowptr) - 1
    row_of = np.repeat(np.arange(rows), np.diff(rowptr))
    kept_rows = row_of[keep]
    rp = np.zeros(rows + 1, np.int64)
    np.add.at(rp, kept_rows + 1, 1)
    return np.cumsum(rp), col[keep], val[keep]


def trial_matrix(g, params, R, Cext, W, s):
    """Sparsifier matrix of one trial from per-length channel counts (the
    batched search reading): with the channel pass's lengths drawn from
    pi = params["s"] (normalised), sum_r (s_r / pi_r) W_r estimates the
    trial's own counts for any pi that is positive wherever s is; then
    Eq. (1)'s truncated logarithm.  Returns a dense-structure FP64 CSR over
    the union of lengths with log x where x > 1 and explicit zeros elsewhere."""
    T = params["T"]
    s = np.asarray(s, np.float64)
    s = s / s.sum()
    pi = np.asarray(params["s"], np.float64)[:T]
    pi = pi / pi.sum()
    if np.any((pi == 0) & (s[:T] > 0)):
        raise ValueError("trial uses a length the channel pass never draws")
    coef = np.where(pi > 0, s[:T] / np.where(pi > 0, pi, 1.0), 0.0)
    rows = np.repeat(np.arange(g.n), np.diff(R))
    base = Cext >> 4
    r = Cext & 15
    key = rows.astype(np.int64) * g.n + base
    uniq, start = np.unique(key, return_index=True)
    grp = np.searchsorted(uniq, key)
    mixed = np.zeros(len(uniq))
    np.add.at(mixed, grp, coef[r] * W.astype(np.float64))
    a = uniq // g.n
    b = uniq % g.n
    assert getattr(g, "weight", None) is None, "channel trials: unweighted graphs"
    deg = degrees(g).astype(np.float64)
    vol = float(volume(g))
    x = vol * vol / (2.0 * params["b"] * params["M"]) / 65536.0 * mixed / (deg[a] * deg[b])
    val = np.where(x > 1.0, np.log(np.where(x > 1.0, x, 1.0)), 0.0)
    rp = np.zeros(g.n + 1, np.int64)
    np.add.at(rp, a + 1, 1)
    return sp.csr_matrix((val, b, np.cumsum(rp)), shape=(g.n, g.n))


def netmf_sparse(g, params, nthreads=None):
    """The sparsified NetMF matrix (FP64 CSR) of the whole graph."""
    R, Cc, W, _, _ = count_csr(g, params, nthreads=nthreads)
    keep, val = trunc_log(g, params, R, Cc, W)
    rp, c2, v2 = compact(R, Cc, keep, val)
    return sp.csr_matrix((v2, c2, rp), shape=(g.n, g.n))


# --------------------------------------------------------------------------
# Randomized SVD (section 4.2)
# --------------------------------------------------------------------------
def gaussian_omega(n: int, k: int, seed: int, rows=None) -> np.ndarray:
    """Omega = randn(n, k) (Algorithm "Fast Randomized SVD", first step), or
    only its rows `rows`.  Entry (i, c) is Box-Muller on the first two words
    of Philox(counter = (i_lo, i_hi, c // 2, TAG_OMEGA)): with u1 =
    (z0+.5)/2^32, u2 = (z1+.5)/2^32, radius sqrt(-2 ln u1), even c takes the
    cosine and odd c the sine of 2 pi u2."""
    half = (k + 1) // 2
    ids = np.arange(n, dtype=np.uint64) if rows is None else np.asarray(rows, dtype=np.uint64)
    n = len(ids)
    i = np.repeat(ids, half)
    c = np.tile(np.arange(half, dtype=np.uint64), n)
    ctr = np.stack([(i & 0xFFFFFFFF).astype(np.uint32), (i >> 32).astype(np.uint32),
                    c.astype(np.uint32), np.full(n * half, TAG_OMEGA, np.uint32)], axis=1)
    z = philox(seed, ctr).astype(np.float64)
    u1 = (z[:, 0] + 0.5) * 2.0 ** -32
    u2 = (z[:, 1] + 0.5) * 2.0 ** -32
    rad = np.sqrt(-2.0 * np.log(u1))
    out = np.empty((n, 2 * half))
    out[:, 0::2] = (rad * np.cos(2.0 * np.pi * u2)).reshape(n, half)
    out[:, 1::2] = (rad * np.sin(2.0 * np.pi * u2)).reshape(n, half)
    return out[:, :k]


def eigsvd(Y: np.ndarray):
    """Algorithm "eigSVD": C = Y^T Y, [V, D] = eig(C), S = sqrt(diag D),
    U = Y V S^-1.  Eigenpairs are sorted by decreasing eigenvalue (the paper's
    LAPACK routine returns them ascending while the top-d columns are used).
    Eigenvalues at or below k * eps * lambda_max are treated as zero and
    their columns of U set to zero."""
    C = Y.T @ Y
    lam, V = np.linalg.eigh(C)
    order = np.argsort(lam)[::-1]
    lam = lam[order]
    V = V[:, order]
    lam = np.where(lam > Y.shape[1] * np.finfo(float).eps * max(lam[0], 0.0), lam, 0.0)
    S = np.sqrt(lam)
    inv = np.where(S > 0, 1.0 / np.where(S > 0, S, 1.0), 0.0)
    U = (Y @ V) * inv
    return U, S, V


def orth_householder(Y: np.ndarray) -> np.ndarray:
    """Orthonormal basis of range(Y) by Householder QR (LAPACK)."""
    Q, _ = np.linalg.qr(Y)
    return Q


def fast_rsvd(M, d: int, oversample: int, q: int, omega: np.ndarray,
              orth: str = "eigsvd"):
    """Algorithm "Fast Randomized SVD" for a symmetric M:
    Y = M Omega; Q = eigSVD(Y).U; q times { Y = M Q; T = Q; [Q, S, V] =
    eigSVD(Y) }; return Q[:, :d], S[:d], T V[:, :d].  ``orth`` replaces the
    orthonormalisation of the power iterations ("householder") for cross
    checks; the final eigSVD is always taken."""
    if q < 1:
        raise ValueError("q >= 1 required (q = 0 leaves S and V undefined)")
    assert omega.shape[1] == d + oversample
    Y = M @ omega
    Q = eigsvd(Y)[0] if orth == "eigsvd" else orth_householder(Y)
    for it in range(q):
        Y = M @ Q
        T = Q
        if it < q - 1 and orth != "eigsvd":
            Q = orth_householder(Y)
            continue
        Q, S, V = eigsvd(Y)
    return Q[:, :d], S[:d], T @ V[:, :d]


def sparse_sign_omega(n: int, k: int, seed: int, rows=None) -> np.ndarray:
    """Sparse-sign test matrix (the alternative to randn(n, k) in the
    randomized SVD): row i has 8 signed unit entries; word t of
    Philox(counter = (i_lo, i_hi, t // 4, TAG_SPARSE_OMEGA)) picks column
    (z >> 1) mod k and sign -1 for odd z, +1 otherwise; entries on one column
    add.  Dense n x k (or only the rows `rows`)."""
    ids = np.arange(n, dtype=np.uint64) if rows is None else np.asarray(rows, dtype=np.uint64)
    n = len(ids)
    out = np.zeros((n, k))
    for b in range(SPARSE_OMEGA_NNZ // 4):
        ctr = np.stack([(ids & 0xFFFFFFFF).astype(np.uint32), (ids >> 32).astype(np.uint32),
                        np.full(n, b, np.uint32), np.full(n, TAG_SPARSE_OMEGA, np.uint32)], axis=1)
        z = philox(seed, ctr).astype(np.uint64)
        for t in range(4):
            c = ((z[:, t] >> 1) % k).astype(np.int64)
            sgn = np.where(z[:, t] & 1, -1.0, 1.0)
            np.add.at(out, (np.arange(n), c), sgn)
    return out


def vanilla_rsvd(M, d: int, oversample: int, q: int, omega: np.ndarray):
    """The vanilla randomized SVD the paper's fast one replaces (section 4.2,
    after Halko, Martinsson and Tropp): Q = an orthonormal basis of M Omega
    (Householder QR), refined by q - 1 subspace iterations Q = qr(M Q); then
    B = Q^T M and its SVD B = U_B S V_B^T give M ~ (Q U_B) S V_B^T.  Returns
    U = Q U_B[:, :d], S[:d], V = V_B[:d]^T.  Same q convention as
    ``fast_rsvd``: q products with M after the first."""
    if q < 1:
        raise ValueError("q >= 1 required")
    Q = orth_householder(M @ omega)
    for _ in range(q - 1):
        Q = orth_householder(M @ Q)
    B = (M.T @ Q).T                       # Q^T M (k' x n)
    Ub, S, Vbt = np.linalg.svd(np.asarray(B), full_matrices=False)
    return Q @ Ub[:, :d], S[:d], Vbt[:d].T


# --------------------------------------------------------------------------
# Spectral propagation (section 4.3)
# --------------------------------------------------------------------------
def cheb_coeffs(theta: float, k: int) -> np.ndarray:
    """Coefficients c_0..c_k of the band-pass filter
    g(lambda) = exp(-theta/2 ((lambda - mu)^2 - 1)) written in Chebyshev
    polynomials T_n(x), x = (lambda - mu)^2 / 2 - 1 (Jacobi-Anger expansion):
    c_0 = e^{-theta/2} I_0(theta), c_n = 2 (-1)^n e^{-theta/2} I_n(theta)."""
    n = np.arange(k + 1)
    c = 2.0 * (-1.0) ** n * scipy.special.iv(n, theta) * math.exp(-theta / 2)
    c[0] /= 2.0
    return c


def _adjacency(g):
    """A as a scipy CSR: arc weights, or ones on an unweighted graph."""
    w = getattr(g, "weight", None)
    data = np.ones(g.n_arcs) if w is None else np.asarray(w, np.float64)
    return sp.csr_matrix((data, g.col, g.rowptr), shape=(g.n, g.n))


def _walk_matrix(g):
    deg = degrees(g).astype(np.float64)
    A = _adjacency(g)
    inv = np.where(deg > 0, 1.0 / np.where(deg > 0, deg, 1.0), 0.0)
    return sp.diags(inv) @ A


def propagate(g, X0: np.ndarray, k: int, theta: float, mu: float) -> np.ndarray:
    """Spectral propagation on the input graph: L = I - D^-1 A, the filter
    g_k(L) = sum_n c_n T_n(L_mu), L_mu = (L - mu I)^2 / 2 - I, applied by the
    Chebyshev three-term recurrence; output D^-1 A (X0 - g_k(L) X0).
    Returns X0 unchanged when k = 0 or theta < 1e-12 (propagation off)."""
    if k == 0 or theta < 1e-12:
        return X0.copy()
    P = _walk_matrix(g)
    c = cheb_coeffs(theta, k)

    def B(Z):
        return (1.0 - mu) * Z - P @ Z      # (L - mu I) Z

    T0 = X0
    T1 = 0.5 * B(B(T0)) - T0
    conv = c[0] * T0 + c[1] * T1
    for nn in range(2, k + 1):
        T2 = B(B(T1)) - 2.0 * T1 - T0
        conv = conv + c[nn] * T2
        T0, T1 = T1, T2
    return P @ (X0 - conv)


def propagate_dense(g, X0: np.ndarray, k: int, theta: float, mu: float,
                    exact: bool = False) -> np.ndarray:
    """Closed form of ``propagate`` through the eigendecomposition of the
    symmetric N = D^-1/2 A D^-1/2: L = D^-1/2 (I - N) D^1/2, so a polynomial
    p(L) = D^-1/2 V p(1 - Lambda) V^T D^1/2.  ``exact`` uses the filter
    g itself instead of its degree-k expansion.  Small graphs only."""
    deg = degrees(g).astype(np.float64)
    A = _adjacency(g).toarray()
    dm = np.where(deg > 0, deg ** -0.5, 0.0)
    N = dm[:, None] * A * dm[None, :]
    lam_n, V = np.linalg.eigh(N)
    lam = 1.0 - lam_n
    x = 0.5 * (lam - mu) ** 2 - 1.0
    if exact:
        gv = np.exp(-0.5 * theta * ((lam - mu) ** 2 - 1.0))
    else:
        c = cheb_coeffs(theta, k)
        gv = np.polynomial.chebyshev.chebval(x, c)
    Dh = np.where(deg > 0, deg ** 0.5, 0.0)
    G = (dm[:, None] * (V * gv) @ V.T) * Dh[None, :]
    P = np.where(deg[:, None] > 0, A / np.where(deg > 0, deg, 1.0)[:, None], 0.0)
    return P @ (X0 - G @ X0)


def bessel_tail_bound(theta: float, k: int) -> float:
    """Sup-norm truncation error of the degree-k expansion on |x| <= 1:
    e^{-theta/2} * 2 * sum_{n > k} I_n(theta)."""
    n = np.arange(k + 1, k + 60)
    return float(math.exp(-theta / 2) * 2.0 * np.sum(scipy.special.iv(n, theta)))


# --------------------------------------------------------------------------
# Whole path
# --------------------------------------------------------------------------
def embedding(U: np.ndarray, S: np.ndarray) -> np.ndarray:
    """X = U S^{1/2} (section 4.2, the embedding from the factorisation)."""
    return U * np.sqrt(S)[None, :]


def final_embedding(Xsp: np.ndarray) -> np.ndarray:
    """eigSVD of the propagated matrix, scaled as X = U_p S_p^{1/2}
    (the last stage of spectral propagation, section 6 time breakdown)."""
    U, S, _ = eigsvd(Xsp)
    return embedding(U, S)


def embed(g, params, nthreads=None, return_stages=False):
    """Sparsified NetMF embedding of graph g (FP64 throughout)."""
    Mmat = netmf_sparse(g, params, nthreads=nthreads)
    d, ov = params["d"], params["oversample"]
    flags = int(params.get("flags", 0))
    omega = (sparse_sign_omega if flags & FLAG_SPARSE_OMEGA else gaussian_omega)(
        g.n, d + ov, params["seed"])
    rsvd = vanilla_rsvd if int(params.get("flags", 0)) & FLAG_VANILLA_RSVD else fast_rsvd
    U, S, V = rsvd(Mmat, d, ov, params["q"], omega)
    X0 = embedding(U, S)
    k, theta, mu = params["cheb_k"], params["theta"], params["mu"]
    if k == 0 or theta < 1e-12:
        X = X0
        Xsp = None
    else:
        Xsp = propagate(g, X0, k, theta, mu)
        X = final_embedding(Xsp)
    if return_stages:
        return dict(M=Mmat, omega=omega, U=U, S=S, V=V, X0=X0, Xsp=Xsp, X=X)
    return X
