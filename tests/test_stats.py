"""The package's time-series statistics on cases with known answers."""
import numpy as np

from paper_1906_06297_amd import stats


def test_binder_limits():
    # a single magnitude (ordered phase): U = 2/3; Gaussian m (disordered): U = 0
    assert abs(stats.binder(np.full(100, 0.7)) - 2.0 / 3.0) < 1e-12
    rng = np.random.default_rng(1)
    assert abs(stats.binder(np.abs(rng.normal(size=400000)))) < 0.01


def test_jackknife_mean_is_standard_error_of_chain_means():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(50, 12)) + rng.normal(size=12)  # chains with their own offsets
    est, se = stats.jackknife_chains(x, np.mean)
    assert abs(est - x.mean()) < 1e-12
    assert abs(se - x.mean(axis=0).std(ddof=1) / np.sqrt(12)) < 1e-12


def test_tau_int_of_an_ar1_process():
    # x_t = phi x_{t-1} + noise: rho(t) = phi^t, tau_int = (1 + phi) / (2 (1 - phi))
    rng = np.random.default_rng(3)
    phi, n, k = 0.8, 20000, 8
    x = np.zeros((n, k))
    e = rng.normal(size=(n, k))
    for t in range(1, n):
        x[t] = phi * x[t - 1] + e[t]
    want = (1 + phi) / (2 * (1 - phi))
    assert abs(stats.tau_int_chains(x) - want) < 0.1 * want
    assert abs(stats.tau_int(x[:, 0]) - want) < 0.25 * want
    # blocking recovers the standard error of a correlated mean: sqrt(2 tau var / n)
    se = stats.blocking_se(x[:, 0])
    assert 0.7 < se / np.sqrt(2 * want * x[:, 0].var() / n) < 1.3
