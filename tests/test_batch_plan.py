"""The batch autotuner's joint choice of tiles (host logic, no GPU): bundles
of every size scheduled longest first on the resident workgroups, and the
choice improved one size at a time for the makespan, then for the sizes'
bundle durations, longest first, then for busy time."""
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


def estimate(lib, opts, pick, slots):
    counts, bundles, ms = _arrays(opts)
    p = (ctypes.c_int * len(opts))(*pick)
    mk, busy = ctypes.c_double(), ctypes.c_double()
    lib.plan_estimate(len(opts), counts, bundles, ms, p, ctypes.c_uint32(slots),
                      ctypes.byref(mk), ctypes.byref(busy))
    return mk.value, busy.value


def choose(lib, opts, start, slots):
    counts, bundles, ms = _arrays(opts)
    s = (ctypes.c_int * len(opts))(*start)
    out = (ctypes.c_int * len(opts))()
    lib.plan_choose(len(opts), counts, bundles, ms, s, ctypes.c_uint32(slots), out)
    return list(out)


def lpt(durations, slots):
    """Longest first, each to the least loaded workgroup."""
    load = [0.0] * slots
    heapq.heapify(load)
    for d in sorted(durations, reverse=True):
        heapq.heappush(load, heapq.heappop(load) + d)
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
    # set by the third size); the first leaves the second size faster
    pick = choose(lib, OPTS, [0, 0, 0], 200)
    assert pick == [1, 0, 0]
    mk, busy = estimate(lib, OPTS, pick, 200)
    assert mk == pytest.approx(20.2)
    assert busy == pytest.approx(48 * 19.1 + 114 * 13.2 + 2 * 20.2)


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
        mk, busy = estimate(lib, opts, list(pick), slots)
        assert mk == pytest.approx(lpt(d, slots))
        assert busy == pytest.approx(sum(d))
        assert mk >= max(d) - 1e-12 and mk >= sum(d) / slots - 1e-12
    def key(pick):
        mk, busy = estimate(lib, opts, pick, slots)
        sizes = sorted((per_bundle(*o[i], slots) for o, i in zip(opts, pick)), reverse=True)
        return (mk, sizes, busy)

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
