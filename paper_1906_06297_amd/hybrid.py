"""Learned global proposals in practice: training data from the plain
checkerboard sampler, training, and hybrid chains that interleave local
bit-packed sweeps with independence Metropolis-Hastings moves proposed by the
autoregressive network.  Every step runs in the library's kernels; this
module only sequences the calls and keeps the bookkeeping.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import lattice as lt


def init_params(L_unused: int, C: int, seed: int, scale: float = 0.5) -> np.ndarray:
    """Random starting parameters in the ABI order (W1, b1, W_l, b_l for
    l = 2..5, W6, b6): normal weights with variance scale^2 * 2 / fan-in,
    zero biases."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, scale * np.sqrt(2 / 4), 4 * C), np.zeros(C)]
    for _ in range(4):
        parts += [rng.normal(0, scale * np.sqrt(2 / (5 * C)), 5 * C * C), np.zeros(C)]
    parts += [rng.normal(0, scale * np.sqrt(1 / (5 * C)), 5 * C), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def plain_configurations(L: int, beta, chains: int, snapshots: int, thin: int, burn: int,
                         seed: int, J: float = 1.0, stream_base: int = 0):
    """(chains * snapshots, L, L) int8 configurations from independent plain
    chains: `burn` sweeps, then a snapshot every `thin` sweeps.  `beta` is one
    inverse temperature, or a sequence that the chains cycle through."""
    betas = np.resize(np.atleast_1d(np.asarray(beta, dtype=np.float64)), chains)
    b = lt.Batch([L] * chains, betas, J, [seed] * chains,
                 list(range(stream_base, stream_base + chains)))
    b.init()
    b.sweep(burn)
    out = torch.empty((snapshots, chains, L, L), dtype=torch.int8, device=b.words.device)
    for k in range(snapshots):
        b.sweep(thin)
        b.spins(out=out[k].view(-1))
    b.close()
    return out.view(-1, L, L)


def train(net: "lt.ARNet", data: torch.Tensor, steps: int, batch: int, lr: float, seed: int = 0,
          log_every: int = 0):
    """Adam on the mean negative log-likelihood of minibatches drawn from
    `data` under random flips and translations (ising_spins_minibatch, step s
    at counter word s)."""
    xb = torch.empty((batch, net.L, net.L), dtype=torch.int8, device=data.device)
    loss = torch.empty(1, dtype=torch.float32, device=data.device)
    hist = []
    for s in range(steps):
        lt.spins_minibatch(data, batch, seed=seed, stream_base=0, round=s, out=xb)
        net.train_step(xb, lr, loss=loss)
        if log_every and (s % log_every == 0 or s == steps - 1):
            hist.append((s, float(loss.item()) / (net.L * net.L)))
    return hist


class Chains:
    """n independent chains on L x L lattices (bit-packed, batch kernel)."""

    def __init__(self, L: int, betas, seed: int, J: float = 1.0, stream_base: int = 0):
        self.L, self.n, self.J = int(L), len(betas), float(J)
        self.betas = np.asarray(betas, dtype=np.float64)
        self.batch = lt.Batch([L] * self.n, self.betas, J, [seed] * self.n,
                              list(range(stream_base, stream_base + self.n)))
        self.batch.init()
        dev = self.batch.words.device
        self.spins = torch.empty((self.n, L, L), dtype=torch.int8, device=dev)
        self.betaJ = torch.as_tensor(self.betas * J, dtype=torch.float32, device=dev)
        self.logq = torch.empty(self.n, dtype=torch.float32, device=dev)
        self.bond = torch.empty(self.n, dtype=torch.int64, device=dev)
        self.mag = torch.empty(self.n, dtype=torch.int64, device=dev)
        self.prop = torch.empty((self.n, L, L), dtype=torch.int8, device=dev)
        self.logq_prop = torch.empty(self.n, dtype=torch.float32, device=dev)
        self.bond_prop = torch.empty(self.n, dtype=torch.int64, device=dev)
        self.mag_prop = torch.empty(self.n, dtype=torch.int64, device=dev)

    def local(self, nsweeps: int) -> None:
        self.batch.sweep(nsweeps)

    def global_move(self, net: "lt.ARNet", seed: int, rnd: int, accepted, stream_base: int = 0):
        """One independence MH move per chain with a fresh proposal from `net`;
        the per-chain decisions (int32, 1 = accepted) go to `accepted`."""
        self.batch.spins(out=self.spins.view(-1))
        net.log_prob(self.spins, out=self.logq)
        lt.spins_observables(self.spins, self.L, bond=self.bond, mag=self.mag)
        net.sample(self.n, seed=seed, stream_base=stream_base, round=rnd, out=self.prop,
                   logq=self.logq_prop)
        lt.spins_observables(self.prop, self.L, bond=self.bond_prop, mag=self.mag_prop)
        lt.mh_independence(self.spins, self.logq, self.bond, self.prop, self.logq_prop,
                           self.bond_prop, self.betaJ, seed=seed + 1, stream_base=stream_base,
                           round=rnd, accepted=accepted)
        self.batch.set_spins(self.spins)

    def close(self):
        self.batch.close()


def run_series(chains: Chains, rounds: int, local_per_round: int, net=None, seed: int = 0,
               round0: int = 1):
    """Per round: `local_per_round` sweeps, then (if net) one global move; the
    observables after each round and the decisions of the moves are written
    by the library straight into per-round device buffers.  Returns (E per
    site, |m|) arrays of shape (rounds, n), the wall time and the number of
    accepted moves per chain (None without a net)."""
    n, N = chains.n, chains.L * chains.L
    dev = chains.spins.device
    obs = torch.empty((rounds, 2, n), dtype=torch.int64, device=dev)
    acc = torch.empty((rounds, n), dtype=torch.int32, device=dev) if net is not None else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in range(rounds):
        if local_per_round:
            chains.local(local_per_round)
        if net is not None:
            chains.global_move(net, seed, round0 + r, accepted=acc[r])
        chains.batch.observables_async(out=obs[r])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    o = obs.cpu().numpy().astype(np.float64)
    E = -chains.J * o[:, 0, :] / N
    A = np.abs(o[:, 1, :]) / N
    accepted = acc.cpu().numpy().sum(axis=0) if acc is not None else None
    return E, A, wall, accepted


def compare_over_betas(net, L: int, betas, per_beta: int, sweeps: int, sweeps_per_proposal: int,
                       burn: int, seed_plain: int, seed_hybrid: int, J: float = 1.0) -> dict:
    """Plain chains against hybrid chains (one global move every
    `sweeps_per_proposal` local sweeps) over a set of temperatures, `per_beta`
    independent chains each, the two kinds seeded independently: per beta the
    energy per site and the Binder cumulant with jackknife errors over chains,
    tau_int(|m|) per measurement, acceptance, and the wall time of both."""
    from . import stats

    betas = np.asarray(betas, dtype=np.float64)
    all_betas = np.repeat(betas, per_beta)
    out = {}
    for kind, use, seed in (("plain", None, seed_plain), ("hybrid", net, seed_hybrid)):
        ch = Chains(L, all_betas, seed=seed, J=J)
        ch.local(burn)
        rounds = sweeps // sweeps_per_proposal
        E, A, wall, acc = run_series(ch, rounds, sweeps_per_proposal, use, seed=seed, round0=1)
        ch.close()
        rows = []
        for k, beta in enumerate(betas):
            cols = slice(k * per_beta, (k + 1) * per_beta)
            e, e_se = stats.jackknife_chains(E[:, cols], np.mean)
            u, u_se = stats.jackknife_chains(A[:, cols], stats.binder)
            rows.append({"beta": float(beta), "E_per_site": e, "E_se": e_se, "binder": u,
                         "binder_se": u_se, "tau_int_abs_m": stats.tau_int_chains(A[:, cols]),
                         "acceptance": (float(acc[cols].sum()) / (per_beta * rounds)
                                        if use is not None else None)})
        out[kind] = {"per_beta": rows, "wall_s": wall, "measurements": rounds}
    return out
