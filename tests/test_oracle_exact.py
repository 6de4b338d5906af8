"""Pins of the exact-physics module against itself by independent routes
(enumeration, transfer matrix, Kaufman, Onsager) and against the paper's T_c."""
import math
import os

import numpy as np
import pytest

from oracle import exact

HERE = os.path.dirname(os.path.abspath(__file__))


def _paper_tc():
    with open(os.path.join(HERE, "golden", "paper_constants.txt")) as f:
        for line in f:
            if line.startswith("Tc_over_J"):
                return float(line.split()[1])


def test_beta_c_matches_paper_tc():
    # Sec. 5.3 quotes T_c = 2.269185 J
    assert abs(1.0 / exact.beta_c() - _paper_tc()) < 5e-7


@pytest.mark.parametrize("beta", [0.2, 0.40, exact.beta_c(), 0.5, 0.9])
def test_enumeration_matches_transfer_matrix_L4(beta):
    e = exact.enumerate_lattice(4, beta)
    t = exact.transfer_matrix(4, beta)
    assert abs(e["E_per_site"] - t["E_per_site"]) < 1e-12


@pytest.mark.parametrize("L", [4, 6, 8])
@pytest.mark.parametrize("beta", [0.25, 0.40, exact.beta_c(), 0.5, 0.7])
def test_kaufman_matches_transfer_matrix(L, beta):
    t = exact.transfer_matrix(L, beta)
    assert abs(exact.kaufman_log_z(beta, L, L) - t["lnZ"]) < 1e-9 * max(1.0, abs(t["lnZ"]))
    assert abs(exact.kaufman_energy(L, beta) - t["E_per_site"]) < 1e-7


@pytest.mark.parametrize("beta", [0.30, 0.40, 0.5, 0.6])
def test_kaufman_tends_to_onsager(beta):
    assert abs(exact.kaufman_energy(512, beta) - exact.onsager_energy(beta)) < 1e-6


def test_onsager_closed_forms():
    # u(beta_c) = -sqrt(2) J; u -> -2J as beta -> inf; u -> 0 as beta -> 0
    assert abs(exact.onsager_energy(exact.beta_c()) + math.sqrt(2)) < 1e-9
    assert abs(exact.onsager_energy(5.0) + 2.0) < 1e-9
    assert abs(exact.onsager_energy(1e-4)) < 1e-3
    # Eq. (7): vanishes at T_c, tends to 1 at T -> 0, zero above T_c
    assert exact.onsager_magnetisation(exact.beta_c() * (1 + 1e-12)) < 0.05
    assert exact.onsager_magnetisation(exact.beta_c() * 0.99) == 0.0
    assert abs(exact.onsager_magnetisation(3.0) - 1.0) < 1e-9


def test_enumeration_symmetries_L4():
    e0 = exact.enumerate_lattice(4, 0.0)
    # infinite temperature: E = 0, <m^2> = 1/N, <m^4> = (3N^2 - 2N)/N^4 for N iid +-1 spins
    N = 16
    assert abs(e0["E_per_site"]) < 1e-15
    assert abs(e0["m2"] - 1.0 / N) < 1e-15
    assert abs(e0["m4"] - (3 * N * N - 2 * N) / N ** 4) < 1e-15
    # ground state limit
    e9 = exact.enumerate_lattice(4, 9.0)
    assert abs(e9["E_per_site"] + 2.0) < 1e-9 and abs(e9["abs_m"] - 1.0) < 1e-9
