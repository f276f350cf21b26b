"""Graph descriptors that condition the hyperparameter search's surrogate
(section 4.4 searches per graph; which statistics describe the graph is this
implementation's reading, R22).  Test infrastructure: only tests/, smoke()
and the benchmark's CPU baseline may import it.

graph_stats(g, seed) returns eight doubles:
  0  log n
  1  log max(m, 1)                        (m undirected edges)
  2  log of the mean degree               (arcs / n)
  3  degree coefficient of variation      (population standard deviation / mean)
  4  log of the maximum degree
  5  Hill tail exponent: 1 + |T| / sum_{d in T} log(d / (x_min - 1/2)),
     x_min = max(1, median degree), T = {degrees >= x_min}
  6  wedge-sampled clustering: the fraction of `wedges` sampled wedges that
     close (wedge_closed below)
  7  spectral gap 1 - lambda_2 of N = D^-1/2 A D^-1/2, lambda_2 estimated by
     `iters` steps of block subspace iteration (spectral_lambda2 below)
Everything is plain FP64 numpy/scipy, written from the definitions; the
random draws are Philox4x32-10 blocks (oracle.philox) and the starting block
is the Gaussian test matrix of the randomized SVD (oracle.gaussian_omega), so
that a device implementation can reproduce them exactly.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .netmf import eigsvd, gaussian_omega, philox

TAG_WEDGE = 6 << 24
BLOCK = 16


def degrees(g) -> np.ndarray:
    return np.diff(np.asarray(g.rowptr, np.int64))


def degree_moments(g):
    """(log n, log max(m, 1), log mean degree, coefficient of variation,
    log max degree) from the degree sequence."""
    d = degrees(g).astype(np.float64)
    n = g.n
    m = len(g.col) // 2
    mean = d.mean()
    return (math.log(n), math.log(max(m, 1)), math.log(mean), d.std() / mean,
            math.log(d.max()))


def hill_exponent(g) -> float:
    """1 + |T| / sum_{d in T} log(d / (x_min - 1/2)), x_min = max(1, median
    degree), T the degrees at or above x_min (a discrete power-law tail
    estimate with the usual half-integer correction)."""
    d = degrees(g).astype(np.float64)
    xmin = max(1.0, float(np.median(d)))
    tail = d[d >= xmin]
    return 1.0 + len(tail) / max(float(np.sum(np.log(tail / (xmin - 0.5)))), 1e-9)


def wedge_closed(g, seed: int, wedges: int) -> int:
    """Number of closed wedges among `wedges` sampled ones.  Wedge t draws the
    Philox block of counter (t_lo, t_hi, 0, 6 << 24) under key `seed`, words
    z0..z3: its centre is candidate ((z1 << 32) | z0) mod C of the C vertices
    of degree >= 2 in increasing order, its ends the neighbours at positions
    a = z2 mod d and b = z3 mod (d - 1), b moved past a when b >= a (two
    distinct neighbours, uniform).  It closes when the ends are adjacent."""
    rp = np.asarray(g.rowptr, np.int64)
    col = np.asarray(g.col, np.int64)
    d = np.diff(rp)
    cand = np.flatnonzero(d >= 2)
    if wedges <= 0 or len(cand) == 0:
        return 0
    t = np.arange(wedges, dtype=np.uint64)
    ctr = np.stack([t & 0xFFFFFFFF, t >> 32, np.zeros_like(t),
                    np.full_like(t, TAG_WEDGE)], axis=1).astype(np.uint32)
    z = philox(seed, ctr).astype(np.uint64)
    closed = 0
    for w in range(wedges):
        c = int(cand[int(((z[w, 1] << np.uint64(32)) | z[w, 0]) % np.uint64(len(cand)))])
        dc = int(d[c])
        ia = int(z[w, 2] % np.uint64(dc))
        ib = int(z[w, 3] % np.uint64(dc - 1))
        if ib >= ia:
            ib += 1
        a, b = int(col[rp[c] + ia]), int(col[rp[c] + ib])
        row = col[rp[a]:rp[a + 1]]
        j = int(np.searchsorted(row, b))
        closed += int(j < len(row) and row[j] == b)
    return closed


def spectral_lambda2(g, seed: int, iters: int, block: int = BLOCK) -> float:
    """lambda_2 of N = D^-1/2 A D^-1/2 (isolated vertices: zero rows) by block
    subspace iteration on M = (I + N) / 2, whose spectrum is that of N moved
    into [0, 1] with the order kept: X = Omega (n x b Gaussian, b = min(16, n),
    key `seed`), then `iters` times Y = M X, [U, S] = eigSVD(Y), X = U; the
    estimate is 2 S_2 - 1 from the last step."""
    n = g.n
    d = degrees(g).astype(np.float64)
    s = np.where(d > 0, 1.0 / np.sqrt(np.where(d > 0, d, 1.0)), 0.0)
    A = sp.csr_matrix((np.ones(len(g.col)), np.asarray(g.col), np.asarray(g.rowptr)),
                      shape=(n, n))
    b = min(block, n)
    X = gaussian_omega(n, b, seed)
    S = np.ones(b)
    for _ in range(iters):
        Y = 0.5 * (X + s[:, None] * (A @ (s[:, None] * X)))
        X, S, _ = eigsvd(Y)
    return 2.0 * float(S[1]) - 1.0 if b > 1 else 2.0 * float(S[0]) - 1.0


def graph_stats(g, seed: int = 0, wedges: int = 2000, iters: int = 200) -> np.ndarray:
    mom = degree_moments(g)
    return np.array(list(mom) + [hill_exponent(g), wedge_closed(g, seed, wedges) / wedges,
                                 1.0 - spectral_lambda2(g, seed, iters)])
