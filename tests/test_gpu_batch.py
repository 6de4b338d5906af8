"""Bit-exact parity of the persistent batch kernel (through the C ABI) with
the CPU oracle on the batched workload, plus counter continuation, batch
invariance, tile invariance and the autotuner."""
import os

import numpy as np
import pytest

import workloads
from layout import pack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    import paper_1906_06297_amd as m

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m.load()
    return m


def say(*a):
    print(*a, flush=True)


def oracle_batch(orc, Ls, betas, J, seeds, streams, nsweeps, ctr=0):
    starts = [orc.init(int(L), int(s), int(q)) for L, s, q in zip(Ls, seeds, streams)]
    if nsweeps == 0:
        return starts
    return orc.batch_sweeps(starts, betas, J, seeds, streams, nsweeps, ctr)


def batch_words_of(batch, q):
    return batch.lattice(q).packed()


@pytest.fixture(scope="module")
def workload():
    Ls, betas, seeds, streams = workloads.batched_lattices()
    return Ls, betas, seeds, streams


@pytest.fixture(scope="module")
def reference_20(orc, workload):
    Ls, betas, seeds, streams = workload
    say("oracle: 1024 lattices x 20 sweeps")
    return oracle_batch(orc, Ls, betas, 1.0, seeds, streams, 20)


def test_batched_workload_20_sweeps(gpu, orc, workload, reference_20):
    Ls, betas, seeds, streams = workload
    say("batch of 1024: init + 20 sweeps")
    b = gpu.Batch(Ls, betas, 1.0, seeds, streams)
    b.init()
    for q in (0, 1, 511, 1023):
        assert np.array_equal(batch_words_of(b, q), pack(orc.init(int(Ls[q]), 3, q)))
    b.sweep(20)
    assert b.counter() == 20
    bad = [q for q in range(len(Ls)) if not np.array_equal(batch_words_of(b, q), pack(reference_20[q]))]
    assert not bad, f"{len(bad)} lattices differ, first {bad[:5]} (L={[int(Ls[q]) for q in bad[:5]]})"
    bond, mag = b.observables()
    for q in range(0, len(Ls), 37):
        assert (int(bond[q]), int(mag[q])) == orc.observables(reference_20[q])
    b.close()


def test_counter_continues_across_graph_replays(gpu, workload, reference_20):
    Ls, betas, seeds, streams = workload
    say("batch: 4 x 5 sweeps")
    b = gpu.Batch(Ls, betas, 1.0, seeds, streams)
    b.init()
    for _ in range(4):
        b.sweep(5)  # the same captured graph, replayed
    assert b.counter() == 20
    for q in range(0, len(Ls), 13):
        assert np.array_equal(batch_words_of(b, q), pack(reference_20[q]))
    b.close()


def test_batch_member_equals_single_lattice(gpu, workload):
    Ls, betas, seeds, streams = workload
    b = gpu.Batch(Ls[:40], betas[:40], 1.0, seeds[:40], streams[:40])
    b.init()
    b.set_counter(7)
    b.sweep(9)
    for q in range(40):
        lone = gpu.Lattice(int(Ls[q]), seed=int(seeds[q]), stream_id=int(streams[q]))
        lone.sweep(float(betas[q]), 1.0, 9, 7)
        assert np.array_equal(lone.packed(), batch_words_of(b, q)), q
    b.close()


@pytest.mark.parametrize("L", [16, 24, 48, 96, 128, 192, 256, 384])
def test_every_tile_gives_the_same_lattice(gpu, orc, L):
    n = 20
    rng = np.random.default_rng(L)
    betas = rng.choice(np.linspace(0.3, 0.6, 32), n)
    Ls = [L] * n
    seeds = [5] * n
    streams = list(range(100, 100 + n))
    ref = oracle_batch(orc, Ls, betas, 1.0, seeds, streams, 6)
    W = (L * L // 2 + 63) // 64
    for lpw in (1, 2):
      for wpt in sorted({1, 2, 3, 4, 6, 8, 16} & set(range(1, W + 1))):
        if -(-W // wpt) * lpw > 1024:
            continue
        say(f"tiles L={L} wpt={wpt} lpw={lpw}")
        b = gpu.Batch(Ls, betas, 1.0, seeds, streams)
        b.set_tiles(L, wpt, lpw)
        assert b.tiles(L) == (wpt, lpw)
        b.init()
        b.sweep(6)
        for q in range(n):
            assert np.array_equal(batch_words_of(b, q), pack(ref[q])), (wpt, lpw, q)
        b.close()


def test_mixed_sizes_and_couplings(gpu, orc):
    Ls = [4, 6, 8, 10, 12, 14, 16, 24, 30, 40, 64, 100, 128, 200, 256, 300, 512, 640]
    n = len(Ls)
    for J in (1.0, -0.7):
        betas = np.linspace(0.0, 0.9, n)
        seeds = [11 + q for q in range(n)]
        streams = [3] * n
        say(f"mixed sizes J={J}")
        b = gpu.Batch(Ls, betas, J, seeds, streams)
        b.init()
        b.sweep(8)
        ref = oracle_batch(orc, Ls, betas, J, seeds, streams, 8)
        for q in range(n):
            assert np.array_equal(batch_words_of(b, q), pack(ref[q])), (J, Ls[q])
        b.close()


def test_mixed_size_bundles_explicit(gpu, orc):
    """Workgroups that mix lattice sizes, tiles and neighbour extractions
    (general, half-word and word rows; one- and two-lane tiles; colours that
    need the refresh): every lattice bit for bit as the oracle."""
    Ls = [16, 24, 30, 64, 100, 128, 192, 256, 40, 64, 14, 192]
    n = len(Ls)
    betas = np.linspace(0.2, 0.7, n)
    seeds = [21 + q for q in range(n)]
    streams = list(range(40, 40 + n))
    say("mixed-size bundles (explicit plan)")
    b = gpu.Batch(Ls, betas, 1.0, seeds, streams)
    b.set_tiles(64, 1, 2)
    b.set_tiles(192, 1, 1)
    b.set_tiles(24, 1, 2)
    b.set_tiles(256, 2, 1)
    b.set_bundles([[7, 0, 1, 4], [6, 3, 2, 9, 10], [5, 11, 8]])
    assert b.mixed()
    b.init()
    b.sweep(8)
    ref = oracle_batch(orc, Ls, betas, 1.0, seeds, streams, 8)
    for q in range(n):
        assert np.array_equal(batch_words_of(b, q), pack(ref[q])), Ls[q]
    # a workgroup's threads and LDS bound what a bundle may hold
    from paper_1906_06297_amd._lib import IsingError
    b.set_tiles(256, 1, 2)  # 1024 threads for one L = 256 lattice
    with pytest.raises(IsingError):
        b.set_bundles([[7, 6], [0, 1, 2, 3, 4, 5, 8, 9, 10, 11]])
    with pytest.raises(IsingError):  # not a permutation
        b.set_bundles([[0, 1], [1, 2]])
    b.close()


def test_long_run_sample(gpu, orc, workload):
    """The workload's full 10^4 sweeps on a sample of its lattices."""
    Ls, betas, seeds, streams = workload
    pick = [q for q in range(len(Ls)) if Ls[q] <= 48][:24]
    sub = [np.asarray(a)[pick] for a in (Ls, betas, seeds, streams)]
    say("batch sample: 24 lattices x 10^4 sweeps")
    b = gpu.Batch(*sub[:2], 1.0, *sub[2:])
    b.init()
    b.sweep(workloads.BATCHED["nsweeps"])
    ref = oracle_batch(orc, *sub[:2], 1.0, *sub[2:], workloads.BATCHED["nsweeps"])
    for i in range(len(pick)):
        assert np.array_equal(batch_words_of(b, i), pack(ref[i])), i
    b.close()


@pytest.mark.timeout(1200)
def test_batched_workload_full_length_every_lattice(gpu, orc, workload, progress):
    """The batched workload as the benchmark runs it -- tiles autotuned for the
    whole batch, 10^4 sweeps in one captured-graph replay from a fresh start --
    every one of the 1024 lattices bit for bit against the oracle (about 1.5e11
    oracle updates: a few minutes on the host's threads)."""
    Ls, betas, seeds, streams = workload
    nsweeps = workloads.BATCHED["nsweeps"]
    b = gpu.Batch(Ls, betas, 1.0, seeds, streams)
    progress("batch of 1024: autotune, then 10^4 sweeps")
    b.autotune(200, None)
    b.init()
    b.set_counter(0)
    b.sweep(nsweeps)
    got = [batch_words_of(b, q) for q in range(len(Ls))]
    assert b.counter() == nsweeps
    b.close()
    progress(f"oracle: 1024 lattices x {nsweeps} sweeps on {orc.max_threads()} threads")
    # in chunks of lattices (each a parallel oracle run), reporting as it goes
    bad = []
    order = np.argsort(-np.asarray(Ls), kind="stable")  # large lattices spread over chunks
    for c in range(16):
        pick = order[c::16]
        ref = oracle_batch(orc, *(np.asarray(a)[pick] for a in (Ls, betas)), 1.0,
                           *(np.asarray(a)[pick] for a in (seeds, streams)), nsweeps)
        bad += [int(q) for k, q in enumerate(pick) if not np.array_equal(got[q], pack(ref[k]))]
        progress(f"  oracle chunk {c + 1}/16 done, {len(bad)} mismatches so far")
    progress(f"{len(Ls) - len(bad)} of {len(Ls)} lattices bit-exact")
    assert not bad, bad[:10]


def test_autotune_keeps_results_and_writes_cache(gpu, orc, tmp_path):
    Ls = [16] * 40 + [96] * 6 + [256] * 3
    n = len(Ls)
    betas = np.linspace(0.35, 0.55, n)
    seeds = [9] * n
    streams = list(range(n))
    path = str(tmp_path / "tiles.json")
    say("autotune")
    b = gpu.Batch(Ls, betas, 1.0, seeds, streams)
    b.init()
    chosen = b.autotune(3, path)
    assert set(chosen) == {16, 96, 256}
    plans = {L: b.plan(L) for L in chosen}
    for L, (per, groups) in plans.items():
        # one size per workgroup fills all but the last; mixed plans may spread them
        assert per >= 1 and groups <= Ls.count(L) <= groups * per, (L, per, groups)
        if not b.mixed():
            assert (groups - 1) * per < Ls.count(L), (L, per, groups)
    assert os.path.exists(path) and "gfx950" in open(path).read()
    b.sweep(5)
    ref = oracle_batch(orc, Ls, betas, 1.0, seeds, streams, 5)
    for q in range(n):
        assert np.array_equal(batch_words_of(b, q), pack(ref[q])), q
    mixed = b.mixed()
    b.close()
    b2 = gpu.Batch(Ls, betas, 1.0, seeds, streams)
    assert b2.autotune(3, path) == chosen  # served from the cache
    assert b2.mixed() == mixed
    assert {L: b2.plan(L) for L in chosen} == plans  # with the lattices per workgroup
    b2.init()
    b2.sweep(5)
    for q in range(n):
        assert np.array_equal(batch_words_of(b2, q), pack(ref[q])), q
    b2.close()
