"""Seeded synthetic graphs standing in for the paper's datasets.

The paper evaluates on public graphs (BlogCatalog ... Hyperlink2014-Sym, see its
dataset table) that are not available here.  These generators produce simple,
undirected, unweighted graphs of the same kinds of shape: planted-block graphs
(stochastic block model) with block labels, and power-law graphs (Chung-Lu,
"erased" multigraph model) optionally with overlapping planted groups.

Output is a symmetric CSR with int64 row offsets and int32 column ids sorted
ascending inside each row, no self-loops and no duplicates.

Numbers come from numpy's PCG64 generator only; torch is used as a sorting
back-end (``device`` may be "cpu" or "cuda"), and every torch operation used
here (unique, sort, scatter-min) is deterministic, so a seed gives the same
graph on every device.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Graph:
    n: int
    rowptr: np.ndarray            # int64, n + 1
    col: np.ndarray               # int32, 2m
    labels: Optional[np.ndarray] = None   # bool n x L (multi-hot) or None
    name: str = ""
    weight: Optional[np.ndarray] = None   # uint32 per arc (symmetric) or None

    @property
    def n_arcs(self) -> int:
        return int(self.rowptr[-1])

    @property
    def m(self) -> int:
        return self.n_arcs // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.rowptr)


def _torch():
    import torch
    return torch


def _first_unique(keys_np: np.ndarray, device: str):
    """Positions of the first occurrence of each distinct key, in draw order."""
    torch = _torch()
    keys = torch.from_numpy(keys_np).to(device)
    uniq, inv = torch.unique(keys, sorted=True, return_inverse=True)
    pos = torch.arange(keys.numel(), device=device, dtype=torch.int64)
    first = torch.full((uniq.numel(),), keys.numel(), device=device,
                       dtype=torch.int64)
    first.scatter_reduce_(0, inv, pos, reduce="amin", include_self=True)
    first, _ = torch.sort(first)
    return first


def _csr_from_pairs(a: np.ndarray, b: np.ndarray, n: int, device: str):
    """Symmetric CSR from undirected pairs a < b (no duplicates)."""
    torch = _torch()
    ta = torch.from_numpy(a.astype(np.int64)).to(device)
    tb = torch.from_numpy(b.astype(np.int64)).to(device)
    rows = torch.cat([ta, tb])
    cols = torch.cat([tb, ta])
    del ta, tb
    key = rows * n + cols
    del rows
    key, _ = torch.sort(key)
    rows = key // n
    cols = (key - rows * n).to(torch.int32)
    del key
    counts = torch.bincount(rows, minlength=n)
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=device)
    rowptr[1:] = torch.cumsum(counts, 0)
    return rowptr.cpu().numpy(), cols.cpu().numpy()


def sbm(sizes, p_in: float, p_out: float, seed: int, device: str = "cpu",
        name: str = "sbm") -> Graph:
    """Exact stochastic block model.

    For every block pair the number of edges is Binomial(#pairs, p) and the
    edge set is a uniform subset of that size, which is the same law as
    independent Bernoulli(p) pairs.  Vertices are numbered block by block and
    the label of a vertex is its block.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = [int(s) for s in sizes]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(off[-1])
    A, B = [], []
    for bi in range(len(sizes)):
        for bj in range(bi, len(sizes)):
            si, sj = sizes[bi], sizes[bj]
            if bi == bj:
                npairs, p = si * (si - 1) // 2, p_in
            else:
                npairs, p = si * sj, p_out
            if npairs == 0 or p <= 0:
                continue
            k = int(rng.binomial(npairs, min(p, 1.0)))
            if k == 0:
                continue
            idx = np.sort(rng.choice(npairs, size=k, replace=False)).astype(np.int64)
            if bi == bj:
                # row-major enumeration of pairs (x, y), x < y inside the block
                # start(x) = x*si - x*(x+1)/2 ; invert with a float guess + fix
                x = np.floor(((2 * si - 1) - np.sqrt((2.0 * si - 1) ** 2 - 8.0 * idx)) / 2).astype(np.int64)
                x = np.clip(x, 0, si - 2)
                start = x * si - x * (x + 1) // 2
                too_big = start > idx
                while np.any(too_big):
                    x[too_big] -= 1
                    start = x * si - x * (x + 1) // 2
                    too_big = start > idx
                nxt = (x + 1) * si - (x + 1) * (x + 2) // 2
                too_small = nxt <= idx
                while np.any(too_small):
                    x[too_small] += 1
                    start = x * si - x * (x + 1) // 2
                    nxt = (x + 1) * si - (x + 1) * (x + 2) // 2
                    too_small = nxt <= idx
                y = idx - start + x + 1
                A.append(off[bi] + x)
                B.append(off[bi] + y)
            else:
                A.append(off[bi] + idx // sj)
                B.append(off[bj] + idx % sj)
    a = np.concatenate(A) if A else np.zeros(0, np.int64)
    b = np.concatenate(B) if B else np.zeros(0, np.int64)
    rowptr, col = _csr_from_pairs(a, b, n, device)
    labels = np.zeros((n, len(sizes)), dtype=bool)
    for bi in range(len(sizes)):
        labels[off[bi]:off[bi + 1], bi] = True
    return Graph(n, rowptr, col, labels, name)


def _cl_offset(n: int, m: int, alpha: float) -> float:
    """Index shift i0 so that vertex 0's expected weight share equals the
    Chung-Lu cap sqrt(2m) (largest expected degree)."""
    target = math.sqrt(2.0 * m)
    beta = 1.0 - alpha

    def deg0(i0):
        z = ((n + i0) ** beta - i0 ** beta) / beta
        w0 = ((1 + i0) ** beta - i0 ** beta) / beta
        return 2.0 * m * w0 / z

    lo, hi = 1e-9, float(n)
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if deg0(mid) > target:
            lo = mid
        else:
            hi = mid
    return hi


def _cl_draw(rng, count: int, n: int, alpha: float, i0: float) -> np.ndarray:
    """Vertex ids with density proportional to (x + i0)^-alpha on [0, n),
    by inverting its closed-form CDF."""
    beta = 1.0 - alpha
    lo = i0 ** beta
    z = (n + i0) ** beta - lo
    u = rng.random(count)
    x = (lo + u * z) ** (1.0 / beta) - i0
    return np.minimum(np.floor(x), n - 1).astype(np.int64)


def chung_lu(n: int, m: int, gamma: float, seed: int, n_groups: int = 0,
             rho: float = 0.7, device: str = "cpu", name: str = "chung_lu") -> Graph:
    """Erased Chung-Lu power-law graph with exactly m undirected edges.

    Endpoints are drawn independently with weight proportional to
    (i + i0)^(-1/(gamma-1)); self-loops and repeated pairs are erased and the
    first m distinct pairs in draw order are kept.  With ``n_groups`` > 0 every
    vertex joins 1-3 distinct groups (uniformly), and each candidate edge is,
    with probability rho, drawn inside one group (group chosen proportionally
    to its size, endpoints by weight inside it); labels are the groups.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    alpha = 1.0 / (gamma - 1.0)
    i0 = _cl_offset(n, m, alpha)
    groups = None
    members = None
    if n_groups > 0:
        k = rng.integers(1, 4, size=n)
        labels = np.zeros((n, n_groups), dtype=bool)
        for i in range(n):
            labels[i, rng.choice(n_groups, size=int(k[i]), replace=False)] = True
        members = [np.flatnonzero(labels[:, g]) for g in range(n_groups)]
        gsize = np.array([len(x) for x in members], dtype=np.float64)
        groups = labels
        # weight of vertex i: integral of the density over [i, i+1)
        beta = 1.0 - alpha
        iw = ((np.arange(n) + 1 + i0) ** beta - (np.arange(n) + i0) ** beta)
        gcdf = [np.cumsum(iw[mb]) / np.sum(iw[mb]) for mb in members]
    draws_a, draws_b = [], []
    total = 0
    batch = int(m * 1.25) + 1024
    while True:
        if groups is None:
            a = _cl_draw(rng, batch, n, alpha, i0)
            b = _cl_draw(rng, batch, n, alpha, i0)
        else:
            inside = rng.random(batch) < rho
            g = rng.choice(n_groups, size=batch, p=gsize / gsize.sum())
            a = _cl_draw(rng, batch, n, alpha, i0)
            b = _cl_draw(rng, batch, n, alpha, i0)
            ua = rng.random(batch)
            ub = rng.random(batch)
            for gi in range(n_groups):
                sel = inside & (g == gi)
                if not np.any(sel):
                    continue
                cdf = gcdf[gi]
                mb = members[gi]
                a[sel] = mb[np.minimum(np.searchsorted(cdf, ua[sel], side="right"), len(mb) - 1)]
                b[sel] = mb[np.minimum(np.searchsorted(cdf, ub[sel], side="right"), len(mb) - 1)]
        draws_a.append(a)
        draws_b.append(b)
        total += batch
        aa = np.concatenate(draws_a)
        bb = np.concatenate(draws_b)
        keep = aa != bb
        lo = np.minimum(aa, bb)[keep]
        hi = np.maximum(aa, bb)[keep]
        keys = lo * n + hi
        first = _first_unique(keys, device)
        if first.numel() >= m:
            take = first[:m].cpu().numpy()
            lo, hi = lo[take], hi[take]
            break
        batch = int(m * 0.25) + 1024
    rowptr, col = _csr_from_pairs(lo, hi, n, device)
    return Graph(n, rowptr, col, groups, name)


def pair_weights(g: Graph, wmax: int, seed: int, device: str = "cpu") -> np.ndarray:
    """Symmetric integer arc weights in 1..wmax: a hash (SplitMix64 finaliser)
    of the seed and the unordered pair, so arcs (u, v) and (v, u) agree.
    Returns uint32 per arc."""
    torch = _torch()
    n = g.n
    rp = torch.from_numpy(np.asarray(g.rowptr, np.int64)).to(device)
    col = torch.from_numpy(np.asarray(g.col, np.int32)).to(device)
    rows = torch.repeat_interleave(torch.arange(n, device=device), rp[1:] - rp[:-1])
    c = col.long()
    key = torch.minimum(rows, c) * n + torch.maximum(rows, c)
    del rows, c

    def srl(x, k):  # logical right shift of int64 bit patterns
        return (x >> k) & ((1 << (64 - k)) - 1)

    z = key + (seed * 0x632BE59BD9B4E019 & 0x7FFFFFFFFFFFFFFF) + 0x1E3779B97F4A7C15
    del key
    z = (z ^ srl(z, 30)) * -4658895280553007687      # 0xBF58476D1CE4E5B9
    z = (z ^ srl(z, 27)) * -7723592293110705685      # 0x94D049BB133111EB
    z = z ^ srl(z, 31)
    w = (srl(z, 1) % wmax + 1).to(torch.int32)
    return w.cpu().numpy().astype(np.uint32)


def relabel(g: Graph, seed: int, device: str = "cpu") -> Graph:
    """g with its vertex ids permuted by a seeded uniform permutation (rows,
    columns, weights and labels alike; neighbour lists sorted again).  The
    generators number vertices in a structured order (Chung-Lu: by expected
    degree); real graphs carry arbitrary ids."""
    torch = _torch()
    n = g.n
    gen = torch.Generator().manual_seed(seed)
    perm = torch.randperm(n, generator=gen).to(device)          # new id of vertex v
    rp = torch.from_numpy(np.asarray(g.rowptr, np.int64)).to(device)
    rows = torch.repeat_interleave(torch.arange(n, device=device), rp[1:] - rp[:-1])
    key = perm[rows] * n
    del rows
    key += perm[torch.from_numpy(np.asarray(g.col)).to(device).long()]
    key, order = torch.sort(key)
    new_rows = torch.div(key, n, rounding_mode="floor")
    col = (key - new_rows * n).to(torch.int32).cpu().numpy()
    del key
    new_rp = np.zeros(n + 1, np.int64)
    new_rp[1:] = torch.cumsum(torch.bincount(new_rows, minlength=n), 0).cpu().numpy()
    del new_rows
    weight = None
    if g.weight is not None:
        weight = torch.from_numpy(np.asarray(g.weight).astype(np.int64)).to(device)[order]
        weight = weight.to(torch.int64).cpu().numpy().astype(np.uint32)
    del order
    labels = None
    if g.labels is not None:
        inv = torch.argsort(perm).cpu().numpy()                 # old id of new vertex i
        labels = np.asarray(g.labels)[inv]
    return Graph(n, new_rp, col, labels, g.name + f"-relabel{seed}", weight)


def dirichlet_s(T: int, seed: int) -> np.ndarray:
    """Per-length weights s_1..s_T drawn from a flat Dirichlet(1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.dirichlet(np.ones(T))


def trial_vectors(count: int, seed: int, T: int = 10):
    """Hyperparameter trials of the batched search: s ~ Dirichlet(1),
    k ~ U{1..20}, theta ~ U[0,1], mu ~ U[0,0.5]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        s = rng.dirichlet(np.ones(T))
        k = int(rng.integers(1, 21))
        theta = float(rng.random())
        mu = float(0.5 * rng.random())
        out.append({"s": s, "k": k, "theta": theta, "mu": mu})
    return out


# Workload catalogue.  Sizes follow the benchmark configurations: a tiny
# planted-block graph, a mid power-law graph with overlapping groups, a large
# power-law one-GPU share, a large planted-block precision case and a batched
# search graph.
WORKLOADS = {
    "tiny": dict(kind="sbm", sizes=[100] * 10, p_in=0.15, p_out=0.005, seed=0,
                 T=10, s="uniform", M_per_Tm=100, d=32, oversample=10, q=1,
                 cheb_k=10, theta=0.5, mu=0.2, precision="f64"),
    "mid": dict(kind="chung_lu", n=10_000, m=330_000, gamma=2.2, groups=39,
                seed=0, T=10, s="dirichlet", M_per_Tm=2000, d=128,
                oversample=10, q=1, cheb_k=10, theta=0.5, mu=0.2,
                precision="f32"),
    "large": dict(kind="chung_lu", n=10_000_000, m=200_000_000, gamma=2.1,
                  groups=0, seed=0, T=5, s=[0.3, 0.7, 0.0, 0.0, 0.0],
                  M_per_Tm=4, d=128, oversample=10, q=1, cheb_k=10,
                  theta=0.5, mu=0.2, precision="f32"),
    "precision": dict(kind="sbm", sizes=[10_000] * 100, p_in=32 / 9_999,
                      p_out=8 / 990_000, seed=0, T=10, s="uniform",
                      M_per_Tm=50, d=256, oversample=10, q=3, cheb_k=10,
                      theta=0.5, mu=0.2, precision="bf16"),
    # intra-block edge share 0.3: the default parameters score a micro-F1 of
    # about 0.46 (10% training labels), inside the unsaturated 0.4-0.8 band
    "batched": dict(kind="sbm", sizes=[2_000] * 50, intra=0.3, avg_deg=30,
                    seed=0, T=10, s="uniform", M_per_Tm=100, d=128,
                    oversample=10, q=1, cheb_k=10, theta=0.5, mu=0.2,
                    precision="f32"),
}


def workload(name: str, device: str = "cpu", **override):
    """(graph, params dict) of a named workload; ``override`` replaces keys."""
    cfg = dict(WORKLOADS[name])
    cfg.update(override)
    if cfg["kind"] == "sbm":
        sizes = cfg["sizes"]
        if "p_in" in cfg:
            p_in, p_out = cfg["p_in"], cfg["p_out"]
        else:
            s0 = sizes[0]
            n = sum(sizes)
            p_in = cfg["intra"] * cfg["avg_deg"] / (s0 - 1)
            p_out = (1 - cfg["intra"]) * cfg["avg_deg"] / (n - s0)
        g = sbm(sizes, p_in, p_out, cfg["seed"], device=device, name=name)
    else:
        g = chung_lu(cfg["n"], cfg["m"], cfg["gamma"], cfg["seed"],
                     n_groups=cfg["groups"], device=device, name=name)
    T = cfg["T"]
    if isinstance(cfg["s"], str):
        s = np.full(T, 1.0 / T) if cfg["s"] == "uniform" else dirichlet_s(T, cfg["seed"])
    else:
        s = np.asarray(cfg["s"], dtype=np.float64)
    params = dict(T=T, s=s, M=int(cfg["M_per_Tm"]) * T * g.m, b=1,
                  C=math.log(g.n), d=cfg["d"], oversample=cfg["oversample"],
                  q=cfg["q"], cheb_k=cfg["cheb_k"], theta=cfg["theta"],
                  mu=cfg["mu"], seed=cfg["seed"], precision=cfg["precision"])
    return g, params
