"""Seeded synthetic workloads for the 2D Ising checkerboard sweep.

This module only draws inputs (sizes, temperatures, seeds, random starting
lattices).  It holds none of the simulation's arithmetic and is shared by the
tests, the benchmark and the smoke check; neither the GPU library nor the CPU
oracle imports it.

Workloads (the paper measures on random +/-1 lattices of given size, Sec. 5.1;
its benchmark temperature and start state are not stated, so these fix them):
  CORRECTNESS  L=64, J=1, beta=0.4406868, seed 42, 1000 sweeps, per-sweep E, M.
  HEADLINE     L=65536 (2^32 spins, 1 bit/spin = 512 MiB), J=1,
               beta in {0.40, 0.4406868, 0.50}, seed 7, 200 sweeps per beta from
               a fresh start; the paper's Table 2 row (32x2048)^2 is this size.
  BATCHED      1024 independent lattices, L uniform over the nine sizes
               {16,24,32,48,64,96,128,192,256} (roughly log-spaced), beta uniform
               over 32 values linspace(0.30, 0.60), drawn with numpy
               default_rng(3); lattice q has stream id q and seed 3; 10^4 sweeps.
"""
from __future__ import annotations

import numpy as np

BETA_CRIT_CONFIG = 0.4406868  # the critical-point coupling as written in the workload

CORRECTNESS = dict(name="correctness", L=64, J=1.0, beta=BETA_CRIT_CONFIG, seed=42, stream=0,
                   nsweeps=1000, rng_counter=0)

HEADLINE = dict(name="headline", L=65536, J=1.0, betas=(0.40, BETA_CRIT_CONFIG, 0.50), seed=7,
                stream=0, nsweeps=200)

BATCH_SIZES = (16, 24, 32, 48, 64, 96, 128, 192, 256)
BATCHED = dict(name="batched", count=1024, sizes=BATCH_SIZES, beta_lo=0.30, beta_hi=0.60,
               n_betas=32, draw_seed=3, seed=3, J=1.0, nsweeps=10_000)


def batched_lattices(count: int = BATCHED["count"], draw_seed: int = BATCHED["draw_seed"]):
    """(Ls, betas, seeds, stream_ids) of the batched workload, in lattice order."""
    rng = np.random.default_rng(draw_seed)
    Ls = rng.choice(np.array(BATCH_SIZES, dtype=np.int64), size=count)
    beta_grid = np.linspace(BATCHED["beta_lo"], BATCHED["beta_hi"], BATCHED["n_betas"])
    betas = rng.choice(beta_grid, size=count)
    seeds = np.full(count, BATCHED["seed"], dtype=np.uint64)
    streams = np.arange(count, dtype=np.uint32)
    return Ls, betas, seeds, streams


def random_spins(L: int, seed: int, p_up: float = 0.5) -> np.ndarray:
    """An L x L int8 lattice of +1/-1 spins, +1 with probability p_up."""
    rng = np.random.default_rng(seed)
    return np.where(rng.random((L, L)) < p_up, 1, -1).astype(np.int8)


# +-J spin glass on the headline lattices: bond signs drawn with probability
# 1/2 from their own Philox key (coupling_seed), the spins as in the headline.
GLASS = dict(name="glass", L=65536, J=1.0, betas=(0.40, BETA_CRIT_CONFIG, 0.50), seed=7, stream=0,
             coupling_seed=11)
