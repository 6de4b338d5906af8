"""Pins of the oracle's +-J spin glass (the extension named in the paper's
conclusions): reductions to the ferromagnet, exact gauge invariance of the
dynamics, the observables, the coupling generator, detailed balance on the
4x4 lattice and long-run averages against enumeration."""
import itertools
import math

import numpy as np
import pytest

import workloads
from oracle import exact, stats

TWO32 = 1 << 32


def field(s, Jr, Jd):
    """h[i,j] = sum over the four bonds of sign * neighbour (periodic)."""
    return (np.roll(Jd, 1, 0) * np.roll(s, 1, 0) + Jd * np.roll(s, -1, 0)
            + np.roll(Jr, 1, 1) * np.roll(s, 1, 1) + Jr * np.roll(s, -1, 1)).astype(np.int64)


def test_all_ferromagnetic_bonds_is_the_ferromagnet(orc):
    L = 24
    a = orc.init(L, 3, 1)
    b = a.copy()
    one = np.ones((L, L), np.int8)
    orc.glass_sweeps(a, one, one, workloads.BETA_CRIT_CONFIG, 1.0, 3, 1, 6, 2)
    orc.sweeps(b, workloads.BETA_CRIT_CONFIG, 1.0, 3, 1, 6, 2)
    assert np.array_equal(a, b)


def test_all_antiferromagnetic_bonds_is_negative_j(orc):
    L = 24
    a = orc.init(L, 4, 0)
    b = a.copy()
    neg = -np.ones((L, L), np.int8)
    orc.glass_sweeps(a, neg, neg, 0.37, 1.0, 4, 0, 6, 0)
    orc.sweeps(b, 0.37, -1.0, 4, 0, 6, 0)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("L", [4, 10, 32])
def test_gauge_invariance_is_exact(orc, L):
    """tau_i = +-1: spins tau s and bonds tau_i J_ij tau_j give the same a at
    every site, hence the same decisions with the same random numbers."""
    rng = np.random.default_rng(L)
    s = orc.init(L, 8, 2)
    Jr, Jd = orc.glass_couplings(L, 21, 0)
    tau = np.where(rng.random((L, L)) < 0.5, -1, 1).astype(np.int8)
    s2 = (tau * s).astype(np.int8)
    Jr2 = (tau * Jr * np.roll(tau, -1, 1)).astype(np.int8)
    Jd2 = (tau * Jd * np.roll(tau, -1, 0)).astype(np.int8)
    e1 = orc.glass_sweeps(s, Jr, Jd, 0.5, 1.0, 8, 2, 5, 1, trace=True)
    e2 = orc.glass_sweeps(s2, Jr2, Jd2, 0.5, 1.0, 8, 2, 5, 1, trace=True)
    assert np.array_equal(s2, tau * s)
    assert np.array_equal(e1[0], e2[0])  # bond sums are gauge invariant


def test_observables_brute_force(orc):
    for L in (4, 6, 16):
        s = workloads.random_spins(L, L + 1)
        Jr, Jd = orc.glass_couplings(L, 5, 1)
        bond = int((s * (Jd * np.roll(s, -1, 0) + Jr * np.roll(s, -1, 1))).sum())
        assert orc.glass_observables(s, Jr, Jd) == (bond, int(s.astype(np.int64).sum()))
        # each bond once: the field sums count every bond twice
        assert 2 * bond == int((s * field(s, Jr, Jd)).sum())


def test_coupling_generator(orc):
    Jr, Jd = orc.glass_couplings(256, 11, 0)
    for a in (Jr, Jd):
        assert set(np.unique(a)) == {-1, 1}
        assert abs((a < 0).mean() - 0.5) < 0.01
    Jr2, Jd2 = orc.glass_couplings(256, 11, 0)
    assert np.array_equal(Jr, Jr2) and np.array_equal(Jd, Jd2)
    Jr3, _ = orc.glass_couplings(256, 12, 0)
    assert not np.array_equal(Jr, Jr3)
    # the right and down bonds are independent draws
    assert abs(np.mean(Jr.astype(int) * Jd) ) < 0.02


def _glass_boltzmann_4x4(beta, Jr, Jd):
    states = exact.all_states(4).astype(np.int64)
    bond = (states * (Jd[None] * np.roll(states, -1, 1) + Jr[None] * np.roll(states, -1, 2))).sum(axis=(1, 2))
    w = np.exp(beta * (bond - bond.max()))
    return w / w.sum(), bond


@pytest.mark.parametrize("beta", [0.4, 1.0])
def test_detailed_balance_per_colour_4x4(orc, beta):
    L = 4
    Jr, Jd = orc.glass_couplings(L, 31, 0)
    pi, _ = _glass_boltzmann_4x4(beta, Jr, Jd)
    states = exact.all_states(L).astype(np.int64)
    T = orc.thresholds(beta, 1.0).astype(np.float64)
    pacc = np.minimum(1.0, T / TWO32)
    i, j = np.indices((L, L))
    h = np.stack([field(st, Jr, Jd) for st in states])
    a = (4 + states * h) // 2
    for c in (0, 1):
        sites = np.argwhere((i + j) % 2 == c)
        p_site = pacc[a[:, sites[:, 0], sites[:, 1]]]
        sub = ((np.arange(256)[:, None] >> np.arange(8)[None, :]) & 1).astype(bool)
        P = np.prod(np.where(sub[None], p_site[:, None, :], 1 - p_site[:, None, :]), axis=2)
        flipmask = (sub.astype(np.int64) << (sites[:, 0] * L + sites[:, 1])[None, :]).sum(axis=1)
        y = np.arange(states.shape[0])[:, None] ^ flipmask[None, :]
        back = P[y, np.arange(256)[None, :]]
        lhs, rhs = pi[:, None] * P, pi[y] * back
        big = np.maximum(lhs, rhs) > 1e-14
        assert (np.abs(lhs - rhs)[big] / np.maximum(lhs, rhs)[big]).max() < 1e-6


def test_long_run_matches_enumeration_4x4(orc):
    L, N, beta = 4, 16, 0.8
    Jr, Jd = orc.glass_couplings(L, 33, 0)
    pi, bond_all = _glass_boltzmann_4x4(beta, Jr, Jd)
    target = float((pi * bond_all).sum()) / N
    s = orc.init(L, 12)
    bond, _ = orc.glass_sweeps(s, Jr, Jd, beta, 1.0, 12, 0, 200_000, trace=True)
    x = bond[1000:] / N
    assert abs(x.mean() - target) < 4.5 * stats.blocking_se(x), (x.mean(), target)
