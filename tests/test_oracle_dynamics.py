"""Pins of the oracle's sweep: deterministic limits, the one-colour Markov
kernel, detailed and global balance, and long-run averages against exact
results (Sec. 2 rule, Sec. 5.3 validation approach)."""
import math

import numpy as np
import pytest

import workloads
from oracle import exact, stats

TWO32 = 1 << 32


def colour_mask(L):
    i, j = np.indices((L, L))
    return (i + j) & 1


def aligned_count(s):
    """a = number of the four neighbours equal to the site (periodic), by array shifts."""
    nb = [np.roll(s, 1, 0), np.roll(s, -1, 0), np.roll(s, 1, 1), np.roll(s, -1, 1)]
    return sum((n == s).astype(np.int64) for n in nb)


# ------------------------------------------------------------ observables
def test_observables_closed_forms(orc):
    L = 12
    N = L * L
    up = np.ones((L, L), np.int8)
    assert orc.observables(up) == (2 * N, N)
    neel = np.where(colour_mask(L) == 0, 1, -1).astype(np.int8)
    assert orc.observables(neel) == (-2 * N, 0)
    one = up.copy()
    one[3, 7] = -1
    assert orc.observables(one) == (2 * N - 8, N - 2)
    stripes = np.tile(np.where(np.arange(L) % 2 == 0, 1, -1).astype(np.int8), (L, 1))
    assert orc.observables(stripes) == (0, 0)


def test_observables_match_bond_count_random(orc):
    for L in (4, 6, 10, 32):
        s = workloads.random_spins(L, 100 + L)
        # bond sum = (sum over sites of sigma * neighbour sum) / 2 = sum over sites (a - 2)
        assert orc.observables(s)[0] == int((aligned_count(s) - 2).sum())
        assert orc.observables(s)[1] == int(s.astype(np.int64).sum())


# ---------------------------------------------------------- deterministic
@pytest.mark.parametrize("L", [4, 6, 10, 16, 24, 64])
def test_beta_zero_flips_every_spin(orc, L):
    s0 = workloads.random_spins(L, L)
    s = s0.copy()
    orc.sweeps(s, 0.0, 1.0, 5, 0, 1)
    assert np.array_equal(s, -s0)
    orc.sweeps(s, 0.0, 1.0, 5, 0, 1, rng_counter=1)
    assert np.array_equal(s, s0)


@pytest.mark.parametrize("L", [4, 8, 14, 32])
def test_zero_temperature_rule(orc, L):
    # 4 beta J > 32 ln 2: T3 = T4 = 0, so a site flips iff a <= 2 (dE <= 0)
    for seed in range(3):
        s = workloads.random_spins(L, 1000 * L + seed)
        for c in (0, 1):
            before = s.copy()
            a = aligned_count(before)
            T = orc.thresholds(10.0, 1.0)
            assert list(T) == [TWO32, TWO32, TWO32, 0, 0]
            orc.half_sweep(s, c, T, 9, 0, 2 * seed + c)
            on = colour_mask(L) == c
            expect = np.where(on & (a <= 2), -before, before)
            assert np.array_equal(s, expect)


def test_zero_temperature_single_defect(orc):
    L = 16
    s = np.ones((L, L), np.int8)
    orc.sweeps(s, 10.0, 1.0, 1, 0, 3)
    assert np.all(s == 1)
    s[5, 6] = -1  # a = 0 -> flips back in its colour's half-sweep
    orc.sweeps(s, 10.0, 1.0, 1, 0, 1)
    assert np.all(s == 1)


def test_j_zero_flips_everything(orc):
    s0 = workloads.random_spins(8, 5)
    s = s0.copy()
    orc.sweeps(s, 0.8, 0.0, 1, 0, 1)
    assert np.array_equal(s, -s0)


# ----------------------------------------------------- one-colour kernel
def metropolis_p(beta, J, a):
    dE = 2.0 * J * (2 * a - 4)
    return 1.0 if dE <= 0 else math.exp(-beta * dE)


@pytest.mark.parametrize("beta,J", [(workloads.BETA_CRIT_CONFIG, 1.0), (0.25, 1.0), (0.3, -1.0)])
def test_flip_frequencies_match_metropolis(orc, beta, J):
    """From a fixed state, many half-sweeps at different t: each site flips with
    probability min(1, exp(-beta dE)) and sites flip independently."""
    L = 16
    s0 = workloads.random_spins(L, 77)
    a = aligned_count(s0)
    T = orc.thresholds(beta, J)
    c = 1
    on = colour_mask(L) == c
    n = 4000
    flips = np.zeros((n, L, L), bool)
    for t in range(n):
        s = s0.copy()
        orc.half_sweep(s, c, T, 123, 4, 1000 + t)
        flips[t] = s != s0
        assert not np.any(flips[t] & ~on)  # the other colour never moves
    for cls in range(5):
        sel = on & (a == cls)
        if not sel.any():
            continue
        p = metropolis_p(beta, J, cls)
        cnt = flips[:, sel].sum()
        tot = n * sel.sum()
        sd = math.sqrt(max(tot * p * (1 - p), 1e-12))
        assert abs(cnt - tot * p) <= 5 * sd + 1e-9, (cls, cnt / tot, p)
    # independence: pairs of same-colour sites with random acceptance
    rnd = np.argwhere(on & np.isin(a, [cls for cls in range(5) if 0 < metropolis_p(beta, J, cls) < 1]))
    rng = np.random.default_rng(5)
    for _ in range(20):
        (i1, j1), (i2, j2) = rnd[rng.choice(len(rnd), 2, replace=False)]
        f1, f2 = flips[:, i1, j1], flips[:, i2, j2]
        p1, p2 = metropolis_p(beta, J, a[i1, j1]), metropolis_p(beta, J, a[i2, j2])
        both = (f1 & f2).sum()
        sd = math.sqrt(n * p1 * p2 * (1 - p1 * p2))
        assert abs(both - n * p1 * p2) <= 5 * sd


# ---------------------------------------------------------- balance (4x4)
def _colour_kernel_4x4(orc, beta, J, c):
    """P_c as (x index, flip-subset) -> (y index, probability), from T[a]."""
    L = 4
    states = exact.all_states(L)
    nst = states.shape[0]
    T = orc.thresholds(beta, J).astype(np.float64)
    pacc = np.minimum(1.0, T / TWO32)
    sites = np.argwhere(colour_mask(L) == c)  # 8 sites
    # a at each colour-c site for each state
    s = states.astype(np.int64)
    nbsum = np.roll(s, 1, 1) + np.roll(s, -1, 1) + np.roll(s, 1, 2) + np.roll(s, -1, 2)
    a = (4 + s * nbsum) // 2
    p_site = pacc[a[:, sites[:, 0], sites[:, 1]]]  # (nst, 8)
    subsets = np.arange(256)
    sub_bits = ((subsets[:, None] >> np.arange(8)[None, :]) & 1).astype(bool)  # (256, 8)
    logp = np.where(sub_bits[None, :, :], np.log(np.maximum(p_site[:, None, :], 1e-300)),
                    np.log(np.maximum(1 - p_site[:, None, :], 1e-300)))
    prob = np.exp(logp.sum(axis=2))
    prob[np.broadcast_to((p_site[:, None, :] == 0) & sub_bits[None], logp.shape).any(axis=2)] = 0.0
    prob[np.broadcast_to((p_site[:, None, :] == 1) & ~sub_bits[None], logp.shape).any(axis=2)] = 0.0
    # state index bit for site (i, j) is i*L + j; flipping toggles those bits
    flipmask = (sub_bits.astype(np.int64) << (sites[:, 0] * L + sites[:, 1])[None, :]).sum(axis=1)
    y = np.arange(nst)[:, None] ^ flipmask[None, :]
    return y, prob


@pytest.mark.parametrize("beta", [0.40, workloads.BETA_CRIT_CONFIG, 0.5])
def test_detailed_balance_per_colour(orc, beta):
    pi = exact.boltzmann_weights(4, beta)
    for c in (0, 1):
        y, P = _colour_kernel_4x4(orc, beta, 1.0, c)
        assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
        # P(y -> x) uses the same flip subset applied from y
        back = P[y, np.arange(256)[None, :]]
        lhs = pi[:, None] * P
        rhs = pi[y] * back
        rel = np.abs(lhs - rhs) / np.maximum(np.maximum(lhs, rhs), 1e-300)
        big = np.maximum(lhs, rhs) > 1e-14
        assert rel[big].max() < 1e-6


def test_global_balance_full_sweep(orc):
    beta = workloads.BETA_CRIT_CONFIG
    pi = exact.boltzmann_weights(4, beta)
    v = pi.copy()
    for c in (0, 1):
        y, P = _colour_kernel_4x4(orc, beta, 1.0, c)
        nv = np.zeros_like(v)
        np.add.at(nv, y.ravel(), (v[:, None] * P).ravel())
        v = nv
    assert np.abs(v - pi).max() < 1e-8 * pi.max()


# --------------------------------------------------- long-run statistics
@pytest.mark.parametrize("beta", [0.40, workloads.BETA_CRIT_CONFIG, 0.50])
def test_long_run_matches_enumeration_4x4(orc, beta):
    L, N = 4, 16
    s = orc.init(L, 31)
    nsw = 200_000
    bond, mag = orc.sweeps(s, beta, 1.0, 31, 0, nsw, trace=True)
    bond, mag = bond[1000:], mag[1000:]
    ex = exact.enumerate_lattice(L, beta)
    e = -bond / N
    m = mag / N
    for series, target in ((e, ex["E_per_site"]), (np.abs(m), ex["abs_m"]), (m * m, ex["m2"])):
        se = stats.blocking_se(series)
        assert abs(series.mean() - target) < 4.5 * se, (series.mean(), target, se)


@pytest.mark.parametrize("L,beta", [(16, 0.40), (16, 0.46), (32, workloads.BETA_CRIT_CONFIG)])
def test_long_run_matches_kaufman(orc, L, beta):
    s = orc.init(L, 8)
    nsw = 40_000 if L == 16 else 20_000
    bond, _ = orc.sweeps(s, beta, 1.0, 8, 0, nsw, trace=True)
    e = -bond[2000:] / (L * L)
    se = stats.blocking_se(e)
    assert abs(e.mean() - exact.kaufman_energy(L, beta)) < 4.5 * se


def test_spontaneous_magnetisation_eq7(orc):
    """Well below T_c the finite lattice sits at Eq. (7)'s magnetisation."""
    L, beta = 64, 0.50
    s = np.ones((L, L), np.int8)
    _, mag = orc.sweeps(s, beta, 1.0, 17, 0, 6000, trace=True)
    m = np.abs(mag[500:]) / (L * L)
    se = stats.blocking_se(m)
    target = exact.onsager_magnetisation(beta)
    # finite-size corrections at L=64, beta=0.5 (xi ~ 1) are far below the error bar
    assert abs(m.mean() - target) < max(4.5 * se, 2e-3), (m.mean(), target, se)


def test_strict_compare_at_equality(orc):
    """The flip needs r < T strictly (Fig. 2 compares the uniform with '<'): a site
    whose uniform equals its threshold stays, one unit above it flips."""
    L, seed, stream, t, c = 16, 99, 2, 37, 0
    s0 = workloads.random_spins(L, 4)
    a = aligned_count(s0)
    sites = np.argwhere((colour_mask(L) == c) & (a >= 3))
    for i, j in sites[:6]:
        n = int(i) * (L // 2) + int(j) // 2
        r = orc.site_uniform(seed, stream, t, n)
        for T_val, should_flip in ((r, False), (r + 1, True)):
            T = np.array([TWO32, TWO32, TWO32, T_val, T_val], dtype=np.uint64)
            s = s0.copy()
            orc.half_sweep(s, c, T, seed, stream, t)
            assert (s[i, j] != s0[i, j]) == should_flip, (i, j, r, T_val)
