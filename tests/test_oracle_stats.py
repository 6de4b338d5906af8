"""Pins of the oracle's time-series statistics (``oracle/stats.py``), which
set the error bars of every statistical test: the autocorrelation estimator
against its direct definition, and tau_int and the blocking standard error
against the closed forms of a first-order autoregressive process,
x_t = phi x_{t-1} + e_t, for which rho(t) = phi^t, tau_int = (1 + phi) /
(2 (1 - phi)) and Var(mean of n) = var(x) / n * (1 + 2 sum_{t<n} (1 - t/n) phi^t)."""
import numpy as np

from oracle import stats


def ar1(phi: float, n: int, k: int, seed: int) -> np.ndarray:
    """k independent stationary AR(1) series of length n, unit innovations."""
    rng = np.random.default_rng(seed)
    e = rng.normal(size=(n, k))
    x = np.empty((n, k))
    x[0] = e[0] / np.sqrt(1.0 - phi * phi)  # stationary start
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    return x


def var_of_mean_ar1(phi: float, n: int) -> float:
    t = np.arange(1, n)
    return (1.0 / (1.0 - phi * phi)) / n * (1.0 + 2.0 * np.sum((1.0 - t / n) * phi ** t))


def test_autocorrelation_is_the_direct_sum():
    x = np.random.default_rng(1).normal(size=300) + 0.3
    d = x - x.mean()
    direct = np.array([np.dot(d[: d.size - t], d[t:]) for t in range(d.size)]) / np.dot(d, d)
    assert np.allclose(stats.autocorrelation(x), direct, atol=1e-12)
    assert np.array_equal(stats.autocorrelation(np.full(10, 2.0)), np.ones(1))


def test_tau_int_of_ar1_processes():
    for phi, seed in ((0.0, 2), (0.5, 3), (0.8, 4), (0.9, 5)):
        want = (1 + phi) / (2 * (1 - phi))
        x = ar1(phi, 8192, 48, seed)
        est = np.array([stats.tau_int(x[:, k]) for k in range(x.shape[1])])
        # Sokal's variance of the windowed estimator, var = 2 (2W + 1) tau^2 / n
        W = 6 * want
        se = np.sqrt(2 * (2 * W + 1) / 8192) * want / np.sqrt(x.shape[1])
        assert abs(est.mean() - want) < 4 * se + 0.02 * want, (phi, est.mean(), want, se)


def test_tau_int_of_an_alternating_series_is_small():
    # rho(t) = (-1)^t (1 - t/n): the window closes at W = 1 with tau = 1/2 - (1 - 1/n)
    x = np.tile([1.0, -1.0], 500)
    assert abs(stats.tau_int(x) - (0.5 - (1 - 1 / 1000))) < 1e-9


def test_blocking_se_of_ar1_processes():
    for phi, seed in ((0.0, 6), (0.6, 7), (0.85, 8)):
        n, k = 1 << 15, 24
        x = ar1(phi, n, k, seed)
        want = np.sqrt(var_of_mean_ar1(phi, n))
        got = np.array([stats.blocking_se(x[:, c]) for c in range(k)])
        # the plateau is the largest level estimate with >= 32 blocks: each is
        # chi-distributed with >= 31 degrees of freedom, and the maximum of a few
        # sits a little above the true value
        r = np.sqrt(np.mean(got ** 2)) / want
        assert 0.9 < r < 1.25, (phi, r)
        # and the spread of the series means agrees with the closed form
        assert 0.7 < x.mean(axis=0).std(ddof=1) / want < 1.3


def test_blocking_se_of_a_constant_and_of_two_values():
    assert stats.blocking_se(np.full(100, 3.0)) == 0.0
    assert np.isnan(stats.blocking_se(np.array([1.0])))
    x = np.array([0.0, 2.0])
    assert abs(stats.blocking_se(x) - np.std(x, ddof=1) / np.sqrt(2)) < 1e-15
