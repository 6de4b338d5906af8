"""Exact results for the periodic 2D Ising model, used to pin the oracle.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Energies follow Eq. (1) with each nearest-neighbour bond counted once:
E = -J * sum_<ij> sigma_i sigma_j, so a periodic L x L lattice has 2 L^2 bonds.

  - ``enumerate_lattice``: brute force over all 2^(L*L) states (L <= 4).
  - ``transfer_matrix``:   row-to-row transfer matrix, exact for L <= 10.
  - ``kaufman_log_z`` / ``kaufman_energy``: Kaufman's closed form for the
    finite periodic lattice (B. Kaufman, Phys. Rev. 76, 1232 (1949); in the
    form of A. E. Ferdinand and M. E. Fisher, Phys. Rev. 185, 832 (1969)).
  - ``onsager_energy``: infinite-lattice energy per site (Onsager 1944, the
    solution the paper validates against, Sec. 5.3).
  - ``onsager_magnetisation``: spontaneous magnetisation, Eq. (7).
  - ``beta_c``: critical coupling from sinh(2 beta_c J) = 1, i.e.
    T_c = 2.269185 J as quoted in Sec. 5.3 (the printed condition
    "tanh(2J/T_c)^2 = 1" has no finite solution; the quoted T_c is that of
    sinh(2J/T_c) = 1).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import ellipk


def beta_c(J: float = 1.0) -> float:
    """Critical inverse temperature: sinh(2 beta J) = 1."""
    return math.log(1.0 + math.sqrt(2.0)) / (2.0 * J)


# ------------------------------------------------------------------ enumeration
def all_states(L: int) -> np.ndarray:
    """All 2^(L*L) configurations as an array (2^(L*L), L, L) of int8 +1/-1."""
    n = L * L
    if n > 20:
        raise ValueError("enumeration is only meant for tiny lattices")
    idx = np.arange(1 << n, dtype=np.int64)
    bits = (idx[:, None] >> np.arange(n)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8).reshape(-1, L, L)


def bond_sum_many(states: np.ndarray) -> np.ndarray:
    """sum_<ij> sigma_i sigma_j for each state (each bond once, periodic)."""
    s = states.astype(np.int64)
    return (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2)) + (s * np.roll(s, -1, axis=2)).sum(axis=(1, 2))


def enumerate_lattice(L: int, beta: float, J: float = 1.0) -> dict:
    """Exact canonical averages by brute force: <E>/N, <|m|>, <m^2>, <m^4>, Binder forms."""
    states = all_states(L)
    N = L * L
    bond = bond_sum_many(states).astype(np.float64)
    M = states.astype(np.int64).sum(axis=(1, 2)).astype(np.float64)
    logw = beta * J * bond  # -beta * E
    logw -= logw.max()
    w = np.exp(logw)
    Z = w.sum()
    m = M / N
    out = {
        "E_per_site": float((w * (-J * bond)).sum() / Z / N),
        "abs_m": float((w * np.abs(m)).sum() / Z),
        "m2": float((w * m ** 2).sum() / Z),
        "m4": float((w * m ** 4).sum() / Z),
    }
    out["binder"] = 1.0 - out["m4"] / (3.0 * out["m2"] ** 2)
    out["binder_as_printed"] = 1.0 - out["m4"] / out["m2"] ** 2
    return out


def boltzmann_weights(L: int, beta: float, J: float = 1.0) -> np.ndarray:
    """Normalised Boltzmann distribution over ``all_states(L)`` order."""
    bond = bond_sum_many(all_states(L)).astype(np.float64)
    logw = beta * J * bond
    logw -= logw.max()
    w = np.exp(logw)
    return w / w.sum()


# -------------------------------------------------------------- transfer matrix
def _row_data(L: int):
    r = np.arange(1 << L, dtype=np.int64)
    spins = 2 * ((r[:, None] >> np.arange(L)[None, :]) & 1) - 1  # (2^L, L)
    intra = (spins * np.roll(spins, -1, axis=1)).sum(axis=1)  # periodic row bonds
    inter = spins @ spins.T  # vertical bonds between two rows
    return spins, intra, inter


def transfer_matrix(L: int, beta: float, J: float = 1.0) -> dict:
    """Exact <E>/N and ln Z of the periodic L x L lattice via the symmetric transfer matrix."""
    if L > 10:
        raise ValueError("transfer matrix is only meant for L <= 10")
    K = beta * J
    _, intra, inter = _row_data(L)
    B = 0.5 * intra[:, None] + 0.5 * intra[None, :] + inter  # bonds attributed to one step
    shift = B.max() * K
    T = np.exp(K * B - shift)
    lam, U = np.linalg.eigh(T)
    # Z = sum_i lam_i^L * exp(L*shift);  d lnZ / dK = L * sum_i lam_i^(L-1) (U^T (B o T) U)_ii / sum lam^L
    dT = B * T
    diag = np.einsum("ji,jk,ki->i", U, dT, U)
    lmax = np.abs(lam).max()
    lr = lam / lmax
    Zr = np.sum(lr ** L)
    dlnZ = L * np.sum(lr ** (L - 1) * diag / lmax) / Zr
    lnZ = math.log(Zr) + L * math.log(lmax) + L * shift
    N = L * L
    return {"lnZ": lnZ, "E_per_site": float(-J * dlnZ / N)}


# --------------------------------------------------------------------- Kaufman
def _signed_log_terms(log_abs: list, signs: list) -> float:
    m = max(log_abs)
    tot = sum(s * math.exp(la - m) for la, s in zip(log_abs, signs))
    if tot <= 0:
        raise ArithmeticError("non-positive partition function")
    return m + math.log(tot)


def kaufman_log_z(K: float, m: int, n: int) -> float:
    """ln Z of an m x n periodic lattice at coupling K = beta*J (Kaufman 1949)."""
    c2, s2 = math.cosh(2 * K), math.sinh(2 * K)
    # gamma_l for l = 0..2n-1:  cosh gamma_l = cosh 2K coth 2K - cos(pi l / n);  gamma_0 = 2K + ln tanh K
    gam = np.empty(2 * n)
    gam[0] = 2 * K + math.log(math.tanh(K))
    ls = np.arange(1, 2 * n)
    gam[1:] = np.arccosh(c2 * c2 / s2 - np.cos(math.pi * ls / n))
    odd = gam[1::2]  # gamma_{2r+1}, r = 0..n-1
    even = gam[0::2]  # gamma_{2r}
    half_m = 0.5 * m

    def log_prod_cosh(g):
        x = half_m * g
        return float(np.sum(np.abs(x) + np.log1p(np.exp(-2 * np.abs(x)))))  # log(2 cosh x)

    def log_prod_sinh(g):
        x = half_m * g
        sign = 1.0
        tot = 0.0
        for v in x:
            if v == 0:
                return float("-inf"), 0.0
            sign *= 1.0 if v > 0 else -1.0
            av = abs(v)
            tot += av + math.log1p(-math.exp(-2 * av))  # log(2 |sinh x|)
        return tot, sign

    l1 = log_prod_cosh(odd)
    l2, s2g = log_prod_sinh(odd)
    l3 = log_prod_cosh(even)
    l4, s4g = log_prod_sinh(even)
    terms, signs = [l1, l3], [1.0, 1.0]
    if s2g != 0.0:
        terms.append(l2)
        signs.append(s2g)
    if s4g != 0.0:
        terms.append(l4)
        signs.append(s4g)
    return math.log(0.5) + 0.5 * m * n * math.log(2 * s2) + _signed_log_terms(terms, signs)


def kaufman_energy(L: int, beta: float, J: float = 1.0, h: float = 2e-4) -> float:
    """Exact <E>/N of the periodic L x L lattice: -J dlnZ/dK / N (Richardson-extrapolated)."""
    K = beta * J

    def d(hh):
        return (kaufman_log_z(K + hh, L, L) - kaufman_log_z(K - hh, L, L)) / (2 * hh)

    dlnZ = (4 * d(h / 2) - d(h)) / 3.0
    return float(-J * dlnZ / (L * L))


# --------------------------------------------------------------------- Onsager
def onsager_energy(beta: float, J: float = 1.0) -> float:
    """Infinite-lattice energy per site, u = -J coth 2K [1 + (2/pi)(2 tanh^2 2K - 1) K1(kappa)]."""
    K = beta * J
    kappa = 2 * math.sinh(2 * K) / math.cosh(2 * K) ** 2
    pre = 2 * math.tanh(2 * K) ** 2 - 1
    m = min(kappa * kappa, 1.0)
    # at the critical point kappa = 1: K1 diverges only logarithmically while
    # the prefactor vanishes linearly, so the product tends to 0
    term = 0.0 if m >= 1.0 else pre * float(ellipk(m))
    return -J / math.tanh(2 * K) * (1 + (2 / math.pi) * term)


def onsager_magnetisation(beta: float, J: float = 1.0) -> float:
    """Eq. (7): (1 - sinh(2J/T)^-4)^(1/8) below T_c, 0 above."""
    x = math.sinh(2 * beta * J)
    if x <= 1.0:
        return 0.0
    return (1.0 - x ** -4) ** 0.125
