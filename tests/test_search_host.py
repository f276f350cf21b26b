"""Host-side logic of the hyperparameter search: the channel-pass length
distribution and the graph statistics fed to the surrogate."""

import numpy as np

from paper_2302_07084_amd import search


def _variance_objective(trials, pi):
    """Sum over trials of sum_r s_r^2 / pi_r: the variance factor of the
    reweighted channel estimate sum_r (s_r / pi_r) W_r."""
    S = np.stack([t.s / t.s.sum() for t in trials])
    return float(np.sum(S ** 2 / pi))


def test_channel_distribution_minimises_the_variance_objective():
    rng = np.random.default_rng(0)
    for _ in range(20):
        trials = search.sample_trials(rng, 16)
        pi = search.channel_distribution(trials, floor=0.0)
        assert abs(pi.sum() - 1) < 1e-12 and np.all(pi > 0)
        best = _variance_objective(trials, pi)
        assert best <= _variance_objective(trials, np.full(10, 0.1)) + 1e-12
        for _ in range(50):                      # and any other distribution
            q = rng.dirichlet(np.ones(10))
            assert best <= _variance_objective(trials, q) + 1e-12


def test_channel_distribution_floor_and_identical_trials():
    t = search.Trial(np.array([0.7, 0.3, 0, 0, 0, 0, 0, 0, 0, 0.0]), 5, 0.5, 0.2)
    pi = search.channel_distribution([t, t], floor=0.1)
    np.testing.assert_allclose(pi, 0.9 * t.s + 0.01)
    assert pi.min() >= 0.01 and abs(pi.sum() - 1) < 1e-12


def test_standardize_is_a_z_score():
    z = search.standardize([1.0, 2.0, 3.0, 4.0])
    assert abs(z.mean()) < 1e-12 and abs(z.std() - 1) < 1e-12
    assert np.all(search.standardize([5.0, 5.0]) == 0)
