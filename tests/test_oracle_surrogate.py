"""Pins of the oracle's surrogate network and scorer."""
import math

import numpy as np
import pytest

from oracle import surrogate as S


def test_gelu_identities():
    x = np.linspace(-6, 6, 101)
    np.testing.assert_allclose(S.gelu(x) - S.gelu(-x), x, atol=1e-14)   # erf is odd
    assert S.gelu(0.0) == 0.0 and abs(S.gelu_grad(0.0) - 0.5) < 1e-15
    np.testing.assert_allclose(S.gelu(np.array([8.0, -8.0])), [8.0, 0.0], atol=1e-12)
    h = 1e-6
    np.testing.assert_allclose(S.gelu_grad(x), (S.gelu(x + h) - S.gelu(x - h)) / (2 * h), atol=1e-8)


@pytest.mark.parametrize("in_dim,h,B", [(3, 4, 5), (21, 16, 9)])
def test_gradient_matches_finite_differences(in_dim, h, B):
    rng = np.random.default_rng(in_dim)
    _, n = S.layout(in_dim, h)
    p = rng.standard_normal(n) * 0.5
    X = rng.standard_normal((B, in_dim))
    t = rng.standard_normal(B)
    _, g = S.loss_and_grad(p, X, t, in_dim, h)
    eps = 1e-6
    num = np.zeros(n)
    for i in range(n):
        e = np.zeros(n)
        e[i] = eps
        num[i] = (S.loss_and_grad(p + e, X, t, in_dim, h)[0] - S.loss_and_grad(p - e, X, t, in_dim, h)[0]) / (2 * eps)
    np.testing.assert_allclose(g, num, rtol=1e-5, atol=1e-8)


def test_adam_first_step_closed_form():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    lr = 0.01
    p1, m, v = S.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr)
    # m_hat = g, v_hat = g^2 at the first step
    np.testing.assert_allclose(p1, p - lr * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_reduces_loss():
    rng = np.random.default_rng(0)
    in_dim, h = 5, 16
    _, n = S.layout(in_dim, h)
    p = rng.standard_normal(n) * 0.3
    X = rng.standard_normal((64, in_dim))
    t = np.sin(X[:, 0]) + 0.5 * X[:, 1]
    m = v = np.zeros(n)
    l0 = S.loss_and_grad(p, X, t, in_dim, h)[0]
    for step in range(1, 301):
        _, g = S.loss_and_grad(p, X, t, in_dim, h)
        p, m, v = S.adam_step(p, g, m, v, step, 0.01)
    assert S.loss_and_grad(p, X, t, in_dim, h)[0] < 0.1 * l0


def test_micro_f1_topk_cases():
    Y = np.array([[1, 0, 0], [0, 1, 1], [0, 0, 1]])
    assert S.micro_f1_topk(Y * 2.0 - 1.0, Y) == 1.0
    scores = np.array([[0, 1, 0], [1, 0, 1], [0, 1, 0]], float)
    # row 0: predicts label 1 (wrong); row 1: predicts 0 and 2 (one right);
    # row 2: predicts 1 (wrong) -> TP 1, FP 3, FN 3
    assert abs(S.micro_f1_topk(scores, Y) - 2 / 8) < 1e-15


def test_scorer_separable_and_random():
    rng = np.random.default_rng(1)
    n, L = 600, 4
    lab = rng.integers(0, L, n)
    Y = np.eye(L, dtype=np.int64)[lab]
    centers = rng.standard_normal((L, 8)) * 5
    X = centers[lab] + rng.standard_normal((n, 8)) * 0.1
    tr, te = np.arange(0, n, 2), np.arange(1, n, 2)
    assert S.score_micro_f1(X, Y, tr, te) == 1.0
    Xr = rng.standard_normal((n, 8))
    assert abs(S.score_micro_f1(Xr, Y, tr, te) - 1 / L) < 0.12
