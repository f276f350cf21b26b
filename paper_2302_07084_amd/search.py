"""Hyperparameter search driven by a learned surrogate (section 4.4).

The paper searches s_1..s_T, M, q and the propagation parameters (k, theta,
mu) with FLAML against the downstream score.  Here a small MLP, trained on
(hyperparameters, graph statistics) -> micro-F1 pairs produced by the plain
method, ranks candidate trials; the plain method (lne_embed followed by
lne_score_micro_f1, both on the GPU) scores every trial that is actually
proposed, so the surrogate only decides the order in which trials are tried
and the plain method's score decides, with random proposals as the fallback
(a share of every round).  This module only orchestrates: the embedding, the scorer and the
network's forward, backward and Adam steps are library kernels.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import (Batch, Context, embed, graph_stats, mlp_adam, mlp_forward, mlp_grad, mlp_init,
               mlp_param_count, score_micro_f1)

T_MAX = 10
N_STATS = 8
IN_DIM = T_MAX + 3 + N_STATS      # s_1..s_10, k, theta, mu, graph statistics
HIDDEN = 256


@dataclasses.dataclass
class Trial:
    s: np.ndarray      # T weights, sum 1
    k: int             # propagation order, 1..20
    theta: float       # [0, 1]
    mu: float          # [0, 0.5]

    def as_dict(self) -> dict:
        return {"s": np.asarray(self.s, np.float64), "k": self.k, "theta": self.theta, "mu": self.mu}

    def vector(self) -> np.ndarray:
        s = np.zeros(T_MAX)
        s[:len(self.s)] = self.s
        return np.concatenate([s, [self.k / 20.0, self.theta, 2.0 * self.mu]])


def sample_trials(rng: np.random.Generator, count: int, T: int = T_MAX):
    """The search space of the batched configuration: s ~ Dirichlet(1),
    k ~ U{1..20}, theta ~ U[0, 1], mu ~ U[0, 0.5]."""
    return [Trial(rng.dirichlet(np.ones(T)), int(rng.integers(1, 21)), float(rng.random()),
                  float(0.5 * rng.random())) for _ in range(count)]


class Surrogate:
    """Device-resident MLP surrogate: features -> predicted micro-F1."""

    def __init__(self, ctx: Context, seed: int = 0, hidden: int = HIDDEN):
        import torch
        self.ctx, self.hidden = ctx, hidden
        self.p = mlp_init(ctx, IN_DIM, hidden, seed)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.step = 0
        self.mu = np.zeros(IN_DIM)
        self.sd = np.ones(IN_DIM)
        self.F = np.zeros((0, IN_DIM))
        self.y = np.zeros(0)

    def add(self, F: np.ndarray, y):
        """Appends observed (features, score) pairs to the training set."""
        self.F = np.concatenate([self.F, F])
        self.y = np.concatenate([self.y, np.asarray(y, np.float64)])

    def set_scaler(self, F: np.ndarray):
        self.mu = F.mean(0)
        self.sd = np.where(F.std(0) > 1e-12, F.std(0), 1.0)

    def _x(self, F):
        import torch
        return torch.from_numpy(((F - self.mu) / self.sd).astype(np.float32)).to(self.ctx.device)

    def fit(self, epochs: int = 400, lr: float = 1e-3):
        """Full-batch Adam on every pair seen so far (library kernels)."""
        import torch
        X = self._x(self.F)
        t = torch.from_numpy(np.asarray(self.y, np.float32)).to(self.ctx.device)
        losses = []
        for _ in range(epochs):
            g, loss = mlp_grad(self.ctx, IN_DIM, self.hidden, self.p, X, t)
            self.step += 1
            mlp_adam(self.ctx, self.p, g, self.m, self.v, self.step, lr)
            losses.append(loss)
        return float(losses[-1].item()), float(losses[0].item())

    def predict(self, F: np.ndarray) -> np.ndarray:
        return mlp_forward(self.ctx, IN_DIM, self.hidden, self.p, self._x(F)).cpu().numpy()


@dataclasses.dataclass
class Task:
    """A labelled graph on the device with the fixed part of the parameters."""
    g: object
    rp: object
    col: object
    labels: object
    base: dict
    stats: np.ndarray
    splits: list

    @staticmethod
    def make(ctx: Context, g, base: dict, train_ratio: float = 0.1, n_splits: int = 1,
             seed: int = 0):
        """The graph on the device, its label splits, and its eight descriptors
        (lne_graph_stats: degree moments, Hill tail exponent, wedge clustering,
        spectral gap)."""
        import torch
        rng = np.random.default_rng(seed)
        splits = []
        for _ in range(n_splits):
            perm = rng.permutation(g.n)
            ntr = max(1, int(round(train_ratio * g.n)))
            splits.append((torch.from_numpy(np.sort(perm[:ntr]).astype(np.int32)).cuda(),
                           torch.from_numpy(np.sort(perm[ntr:]).astype(np.int32)).cuda()))
        rp = torch.from_numpy(g.rowptr).cuda()
        col = torch.from_numpy(g.col).cuda()
        return Task(g, rp, col, torch.from_numpy(g.labels.astype(np.uint8)).cuda(), dict(base),
                    graph_stats(ctx, rp, col, seed), splits)


def evaluate(ctx: Context, task: Task, trial: Trial) -> float:
    """The plain method on one trial: embedding, then micro-F1 averaged over
    the task's splits."""
    p = dict(task.base, s=trial.s, T=len(trial.s), cheb_k=trial.k, theta=trial.theta, mu=trial.mu)
    X, _ = embed(ctx, task.rp, task.col, p)
    return float(np.mean([score_micro_f1(ctx, X, task.labels, tr, te) for tr, te in task.splits]))


def standardize(scores) -> np.ndarray:
    """Scores of one graph's trials as z-scores: the surrogate learns the
    relative quality of hyperparameters on a graph, which is what ranking
    candidates for that graph needs."""
    y = np.asarray(scores, np.float64)
    sd = y.std()
    return (y - y.mean()) / (sd if sd > 1e-12 else 1.0)


def evaluate_batch(ctx: Context, task: Task, batch: Batch, trials, graph: bool = True):
    """The batched method on a list of trials: one batch run (shared sampling
    pass, one launch per step for all trials), then batched scoring on every
    split; returns the micro-F1 per trial and split (trials x splits)."""
    X, _ = batch.run([t.as_dict() for t in trials], graph=graph)
    return np.asarray([score_micro_f1(ctx, X, task.labels, tr, te) for tr, te in task.splits]).T


def features(task: Task, trials) -> np.ndarray:
    return np.stack([np.concatenate([t.vector(), task.stats]) for t in trials])


def random_search(ctx, task, budget, rng):
    trials = sample_trials(rng, budget)
    return trials, [evaluate(ctx, task, t) for t in trials]


def surrogate_search(ctx, task, sur: Surrogate, budget, rng, pool: int = 4096,
                     explore: float = 0.25, rounds: int = 4):
    """Proposes `budget` trials in `rounds` rounds: each round ranks a fresh
    pool of random candidates by the surrogate's prediction and takes the best
    (plus a random share for exploration); every proposal is scored by the
    plain method and the surrogate is refitted on what it has seen."""
    tried, scores = [], []
    per = max(1, budget // rounds)
    while len(tried) < budget:
        n = min(per, budget - len(tried))
        cand = sample_trials(rng, pool)
        pred = sur.predict(features(task, cand))
        n_exp = int(round(explore * n))
        best = [cand[i] for i in np.argsort(-pred)[:n - n_exp]]
        pick = best + sample_trials(rng, n_exp)
        for t in pick:
            tried.append(t)
            scores.append(evaluate(ctx, task, t))
        F_task = features(task, tried)
        # refit on the pretraining pairs plus this graph's pairs so far
        sur_F, sur_y = sur.F, sur.y
        sur.add(F_task, standardize(scores))
        sur.fit(epochs=100)
        sur.F, sur.y = sur_F, sur_y
    return tried, scores


def channel_distribution(trials, floor: float = 0.1) -> np.ndarray:
    """Length distribution of the shared sampling pass for a batch of trials.
    Trial t's channel estimate sum_r (s_r / pi_r) W_r has a variance
    proportional to sum_r s_r^2 / pi_r; the pi minimising its sum over the
    batch is pi_r ~ sqrt(mean_t s_tr^2).  A uniform share `floor` keeps every
    length drawn, which bounds the variance of trials far from the batch."""
    S = np.stack([np.asarray(t.s, np.float64) / np.sum(t.s) for t in trials])
    pi = np.sqrt((S ** 2).mean(axis=0))
    pi = pi / pi.sum()
    return (1.0 - floor) * pi + floor / len(pi)


def pretrain_pairs(ctx: Context, tasks, trials_per_graph: int, rng, max_batch: int = 32):
    """(features, per-graph standardised score) pairs for the surrogate from
    batched runs of random trials on each task's graph."""
    F, y = [], []
    for task in tasks:
        b = None
        trials, scores = [], []
        while len(trials) < trials_per_graph:
            chunk = sample_trials(rng, min(max_batch, trials_per_graph - len(trials)),
                                  T=task.base["T"])
            pi = channel_distribution(chunk)
            if b is None:
                b = Batch(ctx, task.rp, task.col, dict(task.base, s=pi),
                          max_trials=min(max_batch, trials_per_graph))
            else:
                b.resample(pi)
            scores.extend(evaluate_batch(ctx, task, b, chunk).mean(axis=1))
            trials.extend(chunk)
        b.close()
        F.append(features(task, trials))
        y.extend(standardize(scores))
    return np.concatenate(F), np.asarray(y)


def plain_sequential_search(ctx: Context, task: Task, trials, clock=time.perf_counter):
    """The plain method, one trial after another (its own sampling pass per
    trial): returns the scores (trials x splits), the time at which each
    trial's score was known, and the embedding-only seconds."""
    import torch
    t0 = clock()
    scores, stamps, embed_s = [], [], 0.0
    for t in trials:
        a = clock()
        p = dict(task.base, s=t.s, T=len(t.s), cheb_k=t.k, theta=t.theta, mu=t.mu)
        X, _ = embed(ctx, task.rp, task.col, p)
        torch.cuda.synchronize()
        embed_s += clock() - a
        scores.append([score_micro_f1(ctx, X, task.labels, tr, te) for tr, te in task.splits])
        stamps.append(clock() - t0)
    return np.asarray(scores), stamps, embed_s


def batched_surrogate_search(ctx: Context, task: Task, sur, budget: int, rng, per_round: int = 16,
                             pool: int = 4096, explore: float = 0.25, graph: bool = True,
                             clock=time.perf_counter):
    """Batched trials proposed by the surrogate: rounds of `per_round` trials,
    each round ranked by the surrogate (plus a random share), one shared
    sampling pass per round with the length distribution fitted to the
    round's trials, the round run as one batch (HIP graph replay) and scored
    in one batched call; the surrogate is refitted on the graph's
    standardised scores after every round.  Returns trials, scores (trials x
    splits), the time each score was known, the embedding-only seconds and the
    set-up seconds (the sampling pass and launch-shape tuning)."""
    import torch
    t0 = clock()
    b = None
    setup = 0.0
    tried, scores, stamps = [], [], []
    embed_s = 0.0
    base_F, base_y = sur.F, sur.y
    while len(tried) < budget:
        n = min(per_round, budget - len(tried))
        cand = sample_trials(rng, pool, T=task.base["T"])
        pred = sur.predict(features(task, cand))
        n_exp = int(round(explore * n))
        pick = [cand[i] for i in np.argsort(-pred)[:n - n_exp]] + \
            sample_trials(rng, n_exp, T=task.base["T"])
        a = clock()
        pi = channel_distribution(pick)
        if b is None:
            b = Batch(ctx, task.rp, task.col, dict(task.base, s=pi), max_trials=per_round)
            setup = clock() - a
        else:
            b.resample(pi)
        X, _ = b.run([t.as_dict() for t in pick], graph=graph)
        torch.cuda.synchronize()
        embed_s += clock() - a
        got = np.asarray([score_micro_f1(ctx, X, task.labels, tr, te)
                          for tr, te in task.splits]).T
        now = clock() - t0
        tried.extend(pick)
        scores.extend(got)
        stamps.extend([now] * len(pick))
        sur.F, sur.y = base_F, base_y
        sur.add(features(task, tried), standardize(np.asarray(scores).mean(axis=1)))
        sur.fit(epochs=100)
    sur.F, sur.y = base_F, base_y
    b.close()
    return tried, np.asarray(scores), stamps, embed_s, setup
