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


ADDITIVE, ROUNDS = 0, 1


def fit(lib, pts, threads, a_default=0.4, model=ROUNDS):
    n = (ctypes.c_uint32 * len(pts))(*[p[0] for p in pts])
    t = (ctypes.c_double * len(pts))(*[p[1] for p in pts])
    a, b = ctypes.c_double(), ctypes.c_double()
    lib.plan_fit_kind(len(pts), n, t, ctypes.c_uint32(threads), model,
                      ctypes.c_double(a_default), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def pack(lib, kinds, items, slots, max_threads=1024, max_lds=8192, model=ROUNDS):
    k = len(kinds)
    arr = lambda typ, v: (typ * len(v))(*v)
    group = (ctypes.c_int * len(items))()
    lib.plan_pack_mixed.restype = ctypes.c_double
    ms = lib.plan_pack_mixed(k, arr(ctypes.c_double, [x[0] for x in kinds]),
                             arr(ctypes.c_double, [x[1] for x in kinds]),
                             arr(ctypes.c_uint32, [x[2] for x in kinds]),
                             arr(ctypes.c_uint32, [x[3] for x in kinds]),
                             arr(ctypes.c_int, [x[4] if len(x) > 4 else 0 for x in kinds]),
                             len(items),
                             arr(ctypes.c_uint32, items), ctypes.c_uint32(slots),
                             ctypes.c_uint32(max_threads), ctypes.c_uint32(max_lds), model,
                             group)
    return ms, list(group)


def simd_waves(threads):
    return (-(-threads // 64) + 3) // 4


def wg_model(kinds, members, model=ROUNDS):
    """The packer's model of one workgroup: max a + max b * SIMD rounds, or
    max a + sum b."""
    a = max(kinds[k][0] for k in members)
    if model == ADDITIVE:
        return a + sum(kinds[k][1] for k in members)
    b = max(kinds[k][1] for k in members)
    return a + b * simd_waves(sum(kinds[k][2] for k in members))


def model_makespan(kinds, items, group, model=ROUNDS):
    wgs = {}
    for i, g in enumerate(group):
        wgs.setdefault(g, []).append(items[i])
    return max(wg_model(kinds, m, model) for m in wgs.values())


def test_fit_recovers_a_line_over_simd_rounds_and_defaults_a_single_point(lib):
    # 128-thread lattices: 2, 4, 8 of them fill 4, 8, 16 wavefronts: 1, 2, 4 SIMD rounds
    a, b = fit(lib, [(2, 0.5), (8, 0.8), (4, 0.6)], 128)
    assert abs(a - 0.4) < 1e-12 and abs(b - 0.1) < 1e-12
    a, b = fit(lib, [(3, 1.2)], 512, a_default=0.3)  # 24 wavefronts: 6 rounds
    assert abs(a - 0.3) < 1e-12 and abs(b - 0.15) < 1e-12
    a, b = fit(lib, [(1, 1.0)], 64, a_default=2.0)  # a at most 0.8 t
    assert abs(a - 0.8) < 1e-12 and abs(b - 0.2) < 1e-12
    a, b = fit(lib, [(4, 1.0), (16, 0.9)], 256)  # noise: b stays positive, a >= 0
    assert b > 0 and a >= 0


def test_mixed_packing_spreads_long_lattices_and_fills_around_them(lib):
    # 4 long lattices (half a workgroup each), 40 short ones, 8 workgroups
    kinds = [(0.4, 0.25, 512, 1000), (0.3, 0.25, 64, 100)]
    items = [0] * 4 + [1] * 40
    ms, group = pack(lib, kinds, items, 8)
    assert min(group) >= 0
    assert len({group[i] for i in range(4)}) == 4  # one long lattice per workgroup
    assert abs(ms - model_makespan(kinds, items, group)) < 1e-12
    # the long ones alone take two SIMD rounds; the 40 short ones on the other
    # four workgroups three (10 wavefronts each), the best there is
    assert abs(ms - (0.3 + 3 * 0.25)) < 1e-12
    for g in set(group):
        members = [items[i] for i in range(len(items)) if group[i] == g]
        assert sum(kinds[k][2] for k in members) <= 1024
        assert sum(kinds[k][3] for k in members) <= 8192


def test_mixed_packing_respects_capacity_and_reports_failure(lib):
    kinds = [(0.4, 0.6, 1024, 100)]
    ms, group = pack(lib, kinds, [0] * 3, 2)
    assert ms < 0 and group == [-1, -1, -1]
    ms, group = pack(lib, kinds, [0] * 2, 2)
    assert sorted(group) == [0, 1] and abs(ms - (0.4 + 0.6 * 4)) < 1e-12
    # LDS is the limit here
    kinds = [(0.1, 0.1, 1, 5000)]
    ms, group = pack(lib, kinds, [0] * 2, 1)
    assert ms < 0


@pytest.mark.parametrize("seed", range(6))
def test_mixed_packing_on_random_batches(lib, seed):
    rng = np.random.default_rng(seed)
    nk = int(rng.integers(1, 6))
    kinds = [(float(rng.uniform(0.2, 0.6)), float(rng.uniform(0.05, 0.4)),
              int(rng.choice([16, 64, 128, 320, 512])), int(rng.integers(16, 3000)))
             for _ in range(nk)]
    items = [int(x) for x in rng.integers(0, nk, size=int(rng.integers(1, 300)))]
    slots = int(rng.integers(8, 64))
    ms, group = pack(lib, kinds, items, slots)
    if ms < 0:
        return
    assert min(group) >= 0 and max(group) < slots
    assert abs(ms - model_makespan(kinds, items, group)) < 1e-9
    for g in set(group):
        members = [items[i] for i in range(len(items)) if group[i] == g]
        assert sum(kinds[k][2] for k in members) <= 1024
        assert sum(kinds[k][3] for k in members) <= 8192
    # never worse than one lattice per workgroup where that is possible
    if len(items) <= slots:
        assert ms <= max(wg_model(kinds, [k]) for k in items) + max(k[1] for k in kinds) * 4 + 1e-9


def test_exclusive_kinds_keep_workgroups_of_their_own(lib):
    # kind 1 exclusive: never beside kind 0 or 2, though that would pack tighter
    kinds = [(0.4, 0.25, 512, 1000, 0), (0.3, 0.25, 64, 100, 1), (0.3, 0.25, 64, 100, 0)]
    items = [0] * 4 + [1] * 12 + [2] * 12
    ms, group = pack(lib, kinds, items, 8)
    assert min(group) >= 0
    for g in set(group):
        ks = {items[i] for i in range(len(items)) if group[i] == g}
        assert 1 not in ks or ks == {1}
    assert abs(ms - model_makespan(kinds, items, group)) < 1e-12
    # two long lattices share a workgroup, the exclusive one takes the other
    kinds = [(0.4, 0.3, 512, 1000, 0), (0.3, 0.25, 64, 100, 1)]
    ms, group = pack(lib, kinds, [0, 0, 1], 2)
    assert group[0] == group[1] != group[2] and abs(ms - (0.4 + 0.3 * 4)) < 1e-9
    # with too few workgroups for the exclusive kind to get its own, no packing
    ms, group = pack(lib, kinds, [0, 0, 0, 1], 2)
    assert ms < 0


def test_additive_fit_and_packing(lib):
    a, b = fit(lib, [(1, 0.5), (4, 0.8), (2, 0.6)], 64, model=ADDITIVE)
    assert abs(a - 0.4) < 1e-12 and abs(b - 0.1) < 1e-12
    a, b = fit(lib, [(3, 1.2)], 64, a_default=0.3, model=ADDITIVE)
    assert abs(a - 0.3) < 1e-12 and abs(b - 0.3) < 1e-12
    kinds = [(0.4, 0.6, 512, 1000), (0.3, 0.05, 64, 100)]
    items = [0] * 4 + [1] * 40
    ms, group = pack(lib, kinds, items, 8, model=ADDITIVE)
    assert len({group[i] for i in range(4)}) == 4
    assert abs(ms - model_makespan(kinds, items, group, ADDITIVE)) < 1e-12
    total = sum(kinds[k][1] for k in items)
    assert ms <= 0.4 + total / 8 + 0.6 + 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_additive_packing_on_random_batches(lib, seed):
    rng = np.random.default_rng(100 + seed)
    nk = int(rng.integers(1, 6))
    kinds = [(float(rng.uniform(0.2, 0.6)), float(rng.uniform(0.01, 0.6)),
              int(rng.choice([16, 64, 128, 320, 512])), int(rng.integers(16, 3000)),
              int(rng.random() < 0.3)) for _ in range(nk)]
    items = [int(x) for x in rng.integers(0, nk, size=int(rng.integers(1, 300)))]
    slots = int(rng.integers(8, 64))
    ms, group = pack(lib, kinds, items, slots, model=ADDITIVE)
    if ms < 0:
        return
    assert abs(ms - model_makespan(kinds, items, group, ADDITIVE)) < 1e-9
    for g in set(group):
        members = [items[i] for i in range(len(items)) if group[i] == g]
        assert sum(kinds[k][2] for k in members) <= 1024
        assert sum(kinds[k][3] for k in members) <= 8192
        ex = {k for k in members if kinds[k][4]}
        assert not ex or set(members) == ex and len(ex) == 1
