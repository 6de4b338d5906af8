"""Statistics for Markov-chain time series: blocking errors and tau_int.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

  - ``blocking_se``: standard error of the mean of a correlated series by
    repeated pairwise blocking (Flyvbjerg and Petersen, J. Chem. Phys. 91,
    461 (1989)); the plateau is taken as the largest estimate among levels
    with at least 32 blocks.
  - ``tau_int``: integrated autocorrelation time with Sokal's automatic
    window (smallest W with W >= c * tau_int(W), c = 6).
"""
from __future__ import annotations

import numpy as np


def blocking_se(x) -> float:
    x = np.asarray(x, dtype=np.float64)
    n = x.size
    if n < 2:
        return float("nan")
    best = x.std(ddof=1) / np.sqrt(n)
    while x.size >= 64:
        m = x.size // 2
        x = 0.5 * (x[: 2 * m : 2] + x[1 : 2 * m : 2])
        se = x.std(ddof=1) / np.sqrt(x.size)
        best = max(best, se)
    return float(best)


def autocorrelation(x) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    x = x - x.mean()
    n = x.size
    f = np.fft.rfft(x, n=2 * n)
    acf = np.fft.irfft(f * np.conj(f))[:n]
    if acf[0] == 0:
        return np.ones(1)
    return acf / acf[0]


def tau_int(x, c: float = 6.0) -> float:
    """Integrated autocorrelation time tau = 1/2 + sum_{t>=1} rho(t), automatic window."""
    rho = autocorrelation(x)
    tau = 0.5
    for W in range(1, rho.size):
        tau += rho[W]
        if W >= c * tau:
            return float(tau)
    return float(tau)
