"""ORACLE -- test infrastructure, not part of the product.

FP64 reference of the link-prediction evaluation used for the very-large
graphs in the experiments section (after PyTorch-BigGraph's protocol): every
held-out edge (u, v) is ranked among its corrupted edges (u, w_1..w_K) by the
inner product of embedding rows; the ranks give mean rank (MR), mean
reciprocal rank (MRR), HITS@k and AUC.

Definitions (plain, per edge i):
  s(a, b)   = sum_c X[a, c] X[b, c]                      (FP64)
  above_i   = #{j : s(u_i, w_ij) >  s(u_i, v_i)}
  ties_i    = #{j : s(u_i, w_ij) == s(u_i, v_i)}
  rank_i    = 1 + above_i                                (ties favour the edge)
  AUC_i     = (K - above_i - ties_i / 2) / K             (Mann-Whitney)
  MR = mean rank_i, MRR = mean 1 / rank_i, HITS@k = mean [rank_i <= k],
  AUC = mean AUC_i.
"""
from __future__ import annotations

import numpy as np


def scores(X, a, b):
    """s(a_t, b_t) for index arrays a, b (any matching shapes), FP64."""
    X = np.asarray(X, dtype=np.float64)
    return np.einsum("...c,...c->...", X[a], X[b])


def rank_counts(X, pos, neg):
    """(above, ties) per held-out edge: corrupted edges scoring strictly above
    and equal to the edge itself."""
    pos = np.asarray(pos)
    neg = np.asarray(neg)
    sp = scores(X, pos[:, 0], pos[:, 1])
    sn = scores(X, pos[:, 0][:, None], neg)
    above = (sn > sp[:, None]).sum(axis=1)
    ties = (sn == sp[:, None]).sum(axis=1)
    return above.astype(np.int64), ties.astype(np.int64)


def metrics(above, ties, K, hits_k=10):
    """MR, MRR, HITS@hits_k and AUC from the per-edge counts."""
    above = np.asarray(above, dtype=np.float64)
    ties = np.asarray(ties, dtype=np.float64)
    rank = 1.0 + above
    return dict(mean_rank=float(rank.mean()), mrr=float((1.0 / rank).mean()),
                hits=float((rank <= hits_k).mean()),
                auc=float(((K - above - 0.5 * ties) / K).mean()))


def link_metrics(X, pos, neg, hits_k=10):
    above, ties = rank_counts(X, pos, neg)
    return metrics(above, ties, np.asarray(neg).shape[1], hits_k), above, ties
