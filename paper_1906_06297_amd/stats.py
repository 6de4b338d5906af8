"""Time-series statistics for reporting Markov-chain efficiency.

tau_int: integrated autocorrelation time 1/2 + sum_t rho(t) with Sokal's
automatic window (the first W with W >= c * tau(W), c = 6); ess: effective
sample count n / (2 tau_int); blocking_se: standard error of the mean by
repeated halving (Flyvbjerg-Petersen), largest estimate over levels with at
least 32 blocks.
"""
from __future__ import annotations

import numpy as np


def _rho(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    x = x - x.mean()
    n = x.size
    spec = np.fft.rfft(x, 2 * n)
    c = np.fft.irfft(spec * np.conj(spec))[:n]
    return c / c[0] if c[0] > 0 else np.ones(1)


def tau_int(x, c: float = 6.0) -> float:
    rho = _rho(x)
    tau = 0.5
    for w in range(1, rho.size):
        tau += rho[w]
        if w >= c * tau:
            break
    return float(max(tau, 0.5))


def tau_int_chains(series: np.ndarray, c: float = 6.0) -> float:
    """tau_int of several independent chains (rows: time, columns: chains),
    from their averaged normalised autocorrelation."""
    s = np.asarray(series, dtype=np.float64)
    rhos = [_rho(s[:, k]) for k in range(s.shape[1]) if s[:, k].std() > 0]
    if not rhos:
        return float("inf")
    rho = np.mean(rhos, axis=0)
    tau = 0.5
    for w in range(1, rho.size):
        tau += rho[w]
        if w >= c * tau:
            break
    return float(max(tau, 0.5))


def blocking_se(x) -> float:
    x = np.asarray(x, dtype=np.float64)
    best = x.std(ddof=1) / np.sqrt(x.size)
    while x.size >= 64:
        x = 0.5 * (x[: x.size // 2 * 2: 2] + x[1: x.size // 2 * 2: 2])
        best = max(best, x.std(ddof=1) / np.sqrt(x.size))
    return float(best)


def binder(abs_m) -> float:
    """Binder cumulant U = 1 - <m^4> / (3 <m^2>^2) of a sample of |m|."""
    a = np.asarray(abs_m, dtype=np.float64)
    m2, m4 = np.mean(a ** 2), np.mean(a ** 4)
    return float(1.0 - m4 / (3.0 * m2 * m2))


def jackknife_chains(series: np.ndarray, estimator) -> tuple:
    """Estimate and jackknife standard error over independent chains (columns of
    `series`, rows: time): the estimator on all chains, and on the chains with
    one left out in turn."""
    s = np.asarray(series, dtype=np.float64)
    k = s.shape[1]
    full = estimator(s.reshape(-1))
    loo = np.array([estimator(np.delete(s, q, axis=1).reshape(-1)) for q in range(k)])
    se = np.sqrt((k - 1) / k * np.sum((loo - loo.mean()) ** 2))
    return float(full), float(se)
