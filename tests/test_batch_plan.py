"""The batch autotuner's joint choice of tiles (host logic, no GPU): bundles
of every size scheduled longest first on the resident workgroups, and the
choice improved one size at a time for the makespan, then for the sum of
the squared workgroup loads, from several starts."""
import ctypes
import heapq
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    so = str(tmp_path_factory.mktemp("plan") / "libplan.so")
    subprocess.run([gxx, "-O2", "-std=c++17", "-fPIC", "-shared",
                    os.path.join(HERE, "batch_plan_shim.cpp"), "-o", so],
                   check=True, capture_output=True)
    return ctypes.CDLL(so)


def _arrays(opts):
    counts = (ctypes.c_int * len(opts))(*[len(o) for o in opts])
    flat = [x for o in opts for x in o]
    bundles = (ctypes.c_uint32 * len(flat))(*[b for b, _ in flat])
    ms = (ctypes.c_double * len(flat))(*[t for _, t in flat])
    return counts, bundles, ms


def estimate(lib, opts, pick, slots, sumsq=False):
    counts, bundles, ms = _arrays(opts)
    p = (ctypes.c_int * len(opts))(*pick)
    mk, busy, sq = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib.plan_estimate(len(opts), counts, bundles, ms, p, ctypes.c_uint32(slots),
                      ctypes.byref(mk), ctypes.byref(busy), ctypes.byref(sq))
    return (mk.value, busy.value, sq.value) if sumsq else (mk.value, busy.value)


def choose(lib, opts, start, slots):
    counts, bundles, ms = _arrays(opts)
    s = (ctypes.c_int * len(opts))(*start)
    out = (ctypes.c_int * len(opts))()
    lib.plan_choose(len(opts), counts, bundles, ms, s, ctypes.c_uint32(slots), out)
    return list(out)


def lpt(durations, slots, loads=False):
    """Longest first, each to the least loaded workgroup."""
    load = [0.0] * slots
    heapq.heapify(load)
    for d in sorted(durations, reverse=True):
        heapq.heappush(load, heapq.heappop(load) + d)
    if loads:
        return load
    return max(load) if durations else 0.0


def per_bundle(b, t, slots):
    return t / max(1, -(-b // slots))


# three sizes, each with (bundles, ms alone): more bundles run faster alone
OPTS = [[(96, 15.6), (48, 19.1)], [(114, 13.2), (38, 20.2)], [(2, 20.2), (1, 22.4)]]


def test_too_many_bundles_run_a_second_round(lib):
    # the fastest tile of each size alone: 212 bundles on 200 workgroups; the
    # 12 left over follow the shortest bundles
    mk, busy = estimate(lib, OPTS, [0, 0, 0], 200)
    assert mk == pytest.approx(13.2 + 13.2)
    assert busy == pytest.approx(96 * 15.6 + 114 * 13.2 + 2 * 20.2)


def test_joint_choice_fits_one_round(lib):
    # halving either of the first two sizes' bundles fits one round (20.2 ms,
    # set by the third size); halving both leaves the least work in all
    pick = choose(lib, OPTS, [0, 0, 0], 200)
    assert pick == [1, 1, 0]
    mk, busy = estimate(lib, OPTS, pick, 200)
    assert mk == pytest.approx(20.2)
    assert busy == pytest.approx(48 * 19.1 + 38 * 20.2 + 2 * 20.2)


def test_stacked_short_bundles_beat_many_fast_ones(lib):
    # 4 workgroups.  Size 0: one 10 ms bundle (fixed).  Size 1: 6 bundles of
    # 3 ms (6 ms alone: two rounds), or 2 of 5 ms.  Six short bundles stack
    # on three workgroups (6 ms each), two longer ones fit beside the 10 ms
    # bundle: the makespan is 10 either way, and the squared loads prefer the
    # second (less work)
    opts = [[(1, 10.0)], [(6, 6.0), (2, 5.0)]]
    pick = choose(lib, opts, [0, 0], 4)
    assert pick == [0, 1]
    mk, busy, sq = estimate(lib, opts, pick, 4, sumsq=True)
    assert (mk, busy) == (pytest.approx(10.0), pytest.approx(20.0))
    assert sq == pytest.approx(sum(x * x for x in lpt([10.0, 5.0, 5.0], 4, loads=True)))


def test_enough_workgroups_keep_the_fastest_tiles(lib):
    opts = [[(10, 5.0), (5, 8.0)], [(20, 4.0), (4, 9.0)]]
    assert choose(lib, opts, [0, 0], 256) == [0, 0]


def test_a_size_alone_over_several_rounds(lib):
    # 600 bundles on 256 workgroups took 3 rounds alone: 3 ms each
    mk, busy = estimate(lib, [[(600, 9.0)]], [0], 256)
    assert busy == pytest.approx(600 * 3.0)
    assert mk == pytest.approx(lpt([3.0] * 600, 256)) == pytest.approx(9.0)


@pytest.mark.parametrize("seed", range(12))
def test_estimate_and_choice_on_random_batches(lib, seed):
    rng = np.random.default_rng(seed)
    slots = int(rng.integers(2, 12))
    opts = [[(int(rng.integers(1, 15)), float(rng.uniform(1, 10))) for _ in range(rng.integers(1, 4))]
            for _ in range(rng.integers(1, 5))]
    for pick in itertools.product(*[range(len(o)) for o in opts]):
        d = [per_bundle(b, t, slots) for (b, t), i in
             ((o[i], i) for o, i in zip(opts, pick)) for _ in range(b)]
        mk, busy, sq = estimate(lib, opts, list(pick), slots, sumsq=True)
        assert mk == pytest.approx(lpt(d, slots))
        assert busy == pytest.approx(sum(d))
        assert sq == pytest.approx(sum(x * x for x in lpt(d, slots, loads=True)))
        assert mk >= max(d) - 1e-12 and mk >= sum(d) / slots - 1e-12
    def key(pick):
        mk, busy, sq = estimate(lib, opts, pick, slots, sumsq=True)
        sizes = sorted((per_bundle(*o[i], slots) for o, i in zip(opts, pick)), reverse=True)
        return (round(mk * 1e6), sq, sizes, busy)

    start = [0] * len(opts)
    pick = choose(lib, opts, start, slots)
    best = key(pick)
    assert best <= key(start)
    # no single change improves it
    for i, o in enumerate(opts):
        for j in range(len(o)):
            trial = list(pick)
            trial[i] = j
            assert not key(trial) < best
