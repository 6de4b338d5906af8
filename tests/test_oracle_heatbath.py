"""Pins of the oracle's heat-bath rule (Sec. 2: a spin flips with probability
e^{-beta dE} / (e^{-beta dE} + 1)): its threshold table against the closed form
in 60-digit arithmetic, the symmetry that makes the new spin independent of the
old one, flip frequencies, detailed balance of the one-colour kernel on the
4x4 lattice, and long-run averages against exact enumeration and Kaufman."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

import workloads
from oracle import exact, stats

TWO32 = 1 << 32


def colour_mask(L):
    i, j = np.indices((L, L))
    return (i + j) & 1


def aligned_count(s):
    nb = [np.roll(s, 1, 0), np.roll(s, -1, 0), np.roll(s, 1, 1), np.roll(s, -1, 1)]
    return sum((n == s).astype(np.int64) for n in nb)


def heatbath_p(beta, J, a):
    """Flip probability of a spin with a aligned neighbours: dE = 2 J sigma nn = 4 J (a - 2)."""
    dE = 4.0 * J * (a - 2)
    return 1.0 / (1.0 + math.exp(beta * dE))


@pytest.mark.parametrize("J", [1.0, -1.0, 0.5])
def test_table_against_closed_form(orc, J):
    getcontext().prec = 60
    for beta in np.linspace(0.0, 3.0, 61):
        T = orc.thresholds(beta, J, "heatbath")
        for a in range(5):
            dE = Decimal(4) * Decimal(J) * Decimal(a - 2)
            x = Decimal(TWO32) / (1 + (Decimal(float(beta)) * dE).exp())
            want = int(x)  # floor of a positive value
            near_integer = abs(x - want) < Decimal("1e-6") or abs(x - want - 1) < Decimal("1e-6")
            assert int(T[a]) == want or near_integer, (beta, a, int(T[a]), str(x))


def test_table_special_values_and_symmetry(orc):
    assert np.all(orc.thresholds(0.0, 1.0, "heatbath") == TWO32 // 2)
    for beta in np.linspace(0.01, 4.0, 40):
        for J in (1.0, -1.0):
            T = orc.thresholds(beta, J, "heatbath").astype(np.int64)
            assert T[2] == TWO32 // 2  # dE = 0: probability 1/2
            # p(dE) + p(-dE) = 1, so the floors add to 2^32 - 1 (or 2^32 when exact)
            for a in range(5):
                assert T[a] + T[4 - a] in (TWO32 - 1, TWO32), (beta, J, a)
            assert np.all(np.diff(T) <= 0) if J > 0 else np.all(np.diff(T) >= 0)


@pytest.mark.parametrize("beta,J", [(workloads.BETA_CRIT_CONFIG, 1.0), (0.3, -1.0)])
def test_new_spin_is_drawn_from_its_conditional(orc, beta, J):
    """Heat bath: after the update a site is +1 with probability
    1 / (1 + e^{-2 beta J h}), h the neighbour sum, whatever it was before."""
    L = 16
    s0 = workloads.random_spins(L, 91)
    T = orc.thresholds(beta, J, "heatbath")
    c = 0
    on = colour_mask(L) == c
    h = (np.roll(s0, 1, 0) + np.roll(s0, -1, 0) + np.roll(s0, 1, 1) + np.roll(s0, -1, 1)).astype(int)
    n = 3000
    plus = np.zeros((L, L), np.int64)
    for t in range(n):
        s = s0.copy()
        orc.half_sweep(s, c, T, 17, 2, 500 + t)
        assert np.array_equal(s[~on], s0[~on])
        plus += s == 1
    for hv in (-4, -2, 0, 2, 4):
        for sv in (-1, 1):
            sel = on & (h == hv) & (s0 == sv)
            if not sel.any():
                continue
            p = 1.0 / (1.0 + math.exp(-2.0 * beta * J * hv))
            tot = n * sel.sum()
            sd = math.sqrt(max(tot * p * (1 - p), 1e-12))
            assert abs(plus[sel].sum() - tot * p) <= 5 * sd + 1e-9, (hv, sv, plus[sel].sum() / tot, p)


def _colour_kernel_4x4(T, c):
    L = 4
    states = exact.all_states(L)
    nst = states.shape[0]
    pacc = np.minimum(1.0, T.astype(np.float64) / TWO32)
    sites = np.argwhere(colour_mask(L) == c)
    s = states.astype(np.int64)
    nbsum = np.roll(s, 1, 1) + np.roll(s, -1, 1) + np.roll(s, 1, 2) + np.roll(s, -1, 2)
    a = (4 + s * nbsum) // 2
    p_site = pacc[a[:, sites[:, 0], sites[:, 1]]]
    sub_bits = ((np.arange(256)[:, None] >> np.arange(8)[None, :]) & 1).astype(bool)
    prob = np.prod(np.where(sub_bits[None, :, :], p_site[:, None, :], 1 - p_site[:, None, :]), axis=2)
    flipmask = (sub_bits.astype(np.int64) << (sites[:, 0] * L + sites[:, 1])[None, :]).sum(axis=1)
    y = np.arange(nst)[:, None] ^ flipmask[None, :]
    return y, prob


@pytest.mark.parametrize("beta", [0.30, workloads.BETA_CRIT_CONFIG, 0.6])
def test_detailed_balance_per_colour(orc, beta):
    pi = exact.boltzmann_weights(4, beta)
    T = orc.thresholds(beta, 1.0, "heatbath")
    for c in (0, 1):
        y, P = _colour_kernel_4x4(T, c)
        assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
        back = P[y, np.arange(256)[None, :]]
        lhs, rhs = pi[:, None] * P, pi[y] * back
        big = np.maximum(lhs, rhs) > 1e-14
        rel = np.abs(lhs - rhs) / np.maximum(np.maximum(lhs, rhs), 1e-300)
        assert rel[big].max() < 1e-6


@pytest.mark.parametrize("beta", [0.40, workloads.BETA_CRIT_CONFIG, 0.50])
def test_long_run_matches_enumeration_4x4(orc, beta):
    L, N = 4, 16
    s = orc.init(L, 37)
    bond, mag = orc.sweeps(s, beta, 1.0, 37, 0, 200_000, trace=True, rule="heatbath")
    bond, mag = bond[1000:], mag[1000:]
    ex = exact.enumerate_lattice(L, beta)
    for series, target in ((-bond / N, ex["E_per_site"]), (np.abs(mag / N), ex["abs_m"])):
        se = stats.blocking_se(series)
        assert abs(series.mean() - target) < 4.5 * se, (series.mean(), target, se)


def test_long_run_matches_kaufman(orc):
    L, beta = 16, 0.42
    s = orc.init(L, 9)
    bond, _ = orc.sweeps(s, beta, 1.0, 9, 0, 40_000, trace=True, rule="heatbath")
    e = -bond[2000:] / (L * L)
    assert abs(e.mean() - exact.kaufman_energy(L, beta)) < 4.5 * stats.blocking_se(e)


def test_metropolis_sweeps_unchanged_by_the_table_path(orc):
    """orc_sweeps_table with the Metropolis table is orc_sweeps."""
    import ctypes

    import oracle

    L = 24
    a = orc.init(L, 5, 1)
    b = a.copy()
    orc.sweeps(a, 0.43, 1.0, 5, 1, 7, 3)
    T = np.ascontiguousarray(orc.thresholds(0.43, 1.0), dtype=np.uint64)
    oracle.lib().orc_sweeps_table(b.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)), L,
                                  T.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), 5, 1, 7, 3,
                                  None, None)
    assert np.array_equal(a, b)
