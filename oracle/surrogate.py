"""ORACLE -- test infrastructure, not part of the product.

FP64 reference of the surrogate network used by the hyperparameter search
(section 4.4) and of the downstream scorer (the node-classification protocol
of the evaluation section: one-vs-rest logistic regression, micro-F1).

MLP in -> h -> h -> 1 with GELU(z) = z Phi(z) (Phi the standard normal CDF),
mean squared error, Adam (Kingma & Ba) with bias correction.  Parameters use
the flat layout W1 (in x h), b1, W2 (h x h), b2, W3 (h), b3.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def layout(in_dim, h):
    sizes = [("W1", in_dim * h), ("b1", h), ("W2", h * h), ("b2", h), ("W3", h), ("b3", 1)]
    off, out = 0, {}
    for name, n in sizes:
        out[name] = (off, n)
        off += n
    return out, off


def unpack(p, in_dim, h):
    lay, _ = layout(in_dim, h)
    g = {k: p[o:o + n] for k, (o, n) in lay.items()}
    return (g["W1"].reshape(in_dim, h), g["b1"], g["W2"].reshape(h, h), g["b2"],
            g["W3"].reshape(h, 1), g["b3"])


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def forward(p, X, in_dim, h):
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, np.float64), in_dim, h)
    Z1 = X @ W1 + b1
    A1 = gelu(Z1)
    Z2 = A1 @ W2 + b2
    A2 = gelu(Z2)
    y = (A2 @ W3)[:, 0] + b3[0]
    return y, (Z1, A1, Z2, A2)


def loss_and_grad(p, X, t, in_dim, h):
    """Mean squared error and its gradient by the chain rule, layer by layer."""
    p = np.asarray(p, np.float64)
    X = np.asarray(X, np.float64)
    W1, b1, W2, b2, W3, b3 = unpack(p, in_dim, h)
    y, (Z1, A1, Z2, A2) = forward(p, X, in_dim, h)
    B = X.shape[0]
    e = y - t
    loss = float(np.mean(e * e))
    dy = 2.0 * e / B
    gW3 = A2.T @ dy
    gb3 = np.array([dy.sum()])
    dZ2 = np.outer(dy, W3[:, 0]) * gelu_grad(Z2)
    gW2 = A1.T @ dZ2
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2.T) * gelu_grad(Z1)
    gW1 = X.T @ dZ1
    gb1 = dZ1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def micro_f1_topk(scores, Y):
    """Each row predicts its top-k labels, k = its true label count (ties by
    label index); micro-F1 = 2 TP / (2 TP + FP + FN)."""
    tp = fp = fn = 0
    for s, y in zip(scores, Y):
        k = int(y.sum())
        order = np.lexsort((np.arange(len(s)), -s))
        pred = np.zeros_like(y, dtype=bool)
        pred[order[:k]] = True
        yt = y.astype(bool)
        tp += int(np.sum(pred & yt))
        fp += int(np.sum(pred & ~yt))
        fn += int(np.sum(~pred & yt))
    return 2 * tp / (2 * tp + fp + fn) if tp + fp + fn else 0.0


def score_micro_f1(X, Y, train, test, C=1.0):
    """One-vs-rest L2 logistic regression (LIBLINEAR through scikit-learn) on
    standardised features; micro-F1 of the top-k prediction on `test`."""
    from sklearn.linear_model import LogisticRegression
    X = np.asarray(X, np.float64)
    Y = np.asarray(Y).astype(np.int64)
    Xtr = X[train]
    mu = Xtr.mean(0)
    sd = Xtr.std(0)
    sd[sd == 0] = 1.0
    Xtr = (Xtr - mu) / sd
    Xte = (X[test] - mu) / sd
    scores = np.zeros((len(test), Y.shape[1]))
    for l in range(Y.shape[1]):
        yl = Y[train, l]
        if yl.min() == yl.max():
            scores[:, l] = 1.0 if yl[0] == 1 else -1.0
            continue
        clf = LogisticRegression(C=C, solver="liblinear")
        clf.fit(Xtr, yl)
        scores[:, l] = clf.decision_function(Xte)
    return micro_f1_topk(scores, Y[test])
