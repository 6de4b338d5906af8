"""The kernels' per-word logic (the device helpers, compiled for the host)
against the oracle, bit for bit, on the CPU: general and row-aligned
geometries, several temperatures and couplings."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads
from layout import pack

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    so = str(tmp_path_factory.mktemp("emu") / "libemu.so")
    subprocess.run([hipcc, "-O2", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
                    "-x", "hip", os.path.join(HERE, "host_emulator.cpp"), "-o", so], check=True,
                   capture_output=True)
    lib = ctypes.CDLL(so)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.emu_init.argtypes = [u64p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32]
    lib.emu_half_sweep.argtypes = [u64p, ctypes.c_int64, ctypes.c_int, u64p, ctypes.c_int,
                                   ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int]
    lib.emu_half_sweep5.argtypes = [u64p, ctypes.c_int64, ctypes.c_int, u64p, ctypes.c_uint64,
                                    ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int]
    lib.emu_block_decision_check.argtypes = [ctypes.c_uint64, ctypes.c_int]
    lib.emu_start_plain_check.argtypes = [ctypes.c_uint64, ctypes.c_int]
    lib.emu_aligned_neighbours_check.argtypes = [ctypes.c_int64, ctypes.c_uint64]
    lib.emu_half_aligned_neighbours_check.argtypes = [ctypes.c_int64, ctypes.c_uint64]
    lib.emu_ext32_neighbours_check.argtypes = [ctypes.c_int64, ctypes.c_uint64]
    lib.emu_xcd_block.argtypes = [ctypes.c_uint32, ctypes.c_uint32]
    lib.emu_xcd_block.restype = ctypes.c_uint32
    lib.emu_philox_fast.argtypes = [ctypes.c_uint32] * 6 + [ctypes.c_int,
                                                           ctypes.POINTER(ctypes.c_uint32)]
    lib.emu_batch_lattice.argtypes = [u64p, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64,
                                      ctypes.c_uint64, u64p]
    return lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def run_emu(emu, orc, L, seed, stream, beta, J, n, ctr, rows):
    W = (L * L // 2 + 63) // 64
    words = np.zeros(2 * W, dtype=np.uint64)
    emu.emu_init(_p(words), L, seed, stream)
    T = np.ascontiguousarray(orc.thresholds(beta, J), dtype=np.uint64)
    for s in range(n):
        for c in (0, 1):
            emu.emu_half_sweep(_p(words), L, c, _p(T), int(J < 0), 2 * (ctr + s) + c, seed, stream, rows)
    return words.reshape(2, W)


@pytest.mark.parametrize("L", [4, 6, 8, 10, 12, 16, 24, 30, 48, 64, 96, 100, 128, 256])
@pytest.mark.parametrize("beta,J", [(0.0, 1.0), (workloads.BETA_CRIT_CONFIG, 1.0), (0.5, 1.0),
                                    (9.0, 1.0), (0.3, -1.0), (0.4, 0.0)])
def test_general_kernel_logic(emu, orc, L, beta, J):
    seed, stream, n, ctr = 77 + L, 5, 4, 3
    ref = orc.init(L, seed, stream)
    w0 = run_emu(emu, orc, L, seed, stream, beta, J, 0, ctr, 0)
    assert np.array_equal(w0, pack(ref))
    orc.sweeps(ref, beta, J, seed, stream, n, ctr)
    assert np.array_equal(run_emu(emu, orc, L, seed, stream, beta, J, n, ctr, 0), pack(ref))


@pytest.mark.parametrize("rows", [1, 2])
@pytest.mark.parametrize("L", [128, 256, 512])
@pytest.mark.parametrize("beta,J", [(0.0, 1.0), (0.40, 1.0), (workloads.BETA_CRIT_CONFIG, 1.0),
                                    (0.5, 1.0), (0.3, -1.0), (7.0, 1.0), (7.0, -1.0),
                                    (0.0, -1.0)])
def test_row_kernel_logic(emu, orc, rows, L, beta, J):
    seed, stream, n, ctr = 7, 0, 3, 0
    ref = orc.init(L, seed, stream)
    orc.sweeps(ref, beta, J, seed, stream, n, ctr)
    assert np.array_equal(run_emu(emu, orc, L, seed, stream, beta, J, n, ctr, rows), pack(ref))


@pytest.mark.parametrize("L", [4, 6, 8, 10, 12, 16, 24, 32, 48, 64, 96, 100, 128, 192, 256])
@pytest.mark.parametrize("beta,J", [(0.0, 1.0), (workloads.BETA_CRIT_CONFIG, 1.0), (0.31, 1.0),
                                    (0.3, -1.0), (5.0, 1.0)])
def test_batch_kernel_logic(emu, orc, L, beta, J):
    """The persistent batch kernel's LDS sequence (extended cyclic colour arrays)."""
    seed, stream, n, ctr = 3, 17, 5, 9
    ref = orc.init(L, seed, stream)
    words = np.ascontiguousarray(pack(ref).reshape(-1))
    T = np.ascontiguousarray(orc.thresholds(beta, J), dtype=np.uint64)
    emu.emu_batch_lattice(_p(words), L, beta, J, seed, stream, n, ctr, _p(T))
    orc.sweeps(ref, beta, J, seed, stream, n, ctr)
    assert np.array_equal(words.reshape(2, -1), pack(ref))


def _kat_rows():
    path = os.path.join(HERE, "golden", "philox4x32_10_kat.txt")
    rows = []
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            v = [int(x, 16) for x in line.split()]
            rows.append((v[:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_fused_xor_philox(emu, orc, mode):
    """The Philox rounds written with three-input XORs give the published
    known answers and the oracle's blocks on random counters and keys."""
    out = (ctypes.c_uint32 * 4)()
    for ctr, key, want in _kat_rows():
        emu.emu_philox_fast(*ctr, *key, mode, out)
        assert list(out) == want
    rng = np.random.default_rng(11)
    for _ in range(2000):
        ctr = [int(x) for x in rng.integers(0, 2 ** 32, 4, dtype=np.uint64)]
        key = [int(x) for x in rng.integers(0, 2 ** 32, 2, dtype=np.uint64)]
        emu.emu_philox_fast(*ctr, *key, mode, out)
        assert tuple(out) == tuple(orc.philox4x32_10(ctr, key))


@pytest.mark.parametrize("n", [1, 7, 8, 9, 15, 16, 17, 255, 256, 4095, 4096, 65536, 65541])
def test_xcd_block_order_is_a_permutation(emu, n):
    got = np.array([emu.emu_xcd_block(b, n) for b in range(n)])
    assert np.array_equal(np.sort(got), np.arange(n))
    # each XCD (b % 8) receives one contiguous range of logical blocks
    for x in range(min(n, 8)):
        mine = np.sort(got[x::8])
        assert np.all(np.diff(mine) == 1)


@pytest.mark.parametrize("L,rows5", [(4, 0), (6, 0), (10, 0), (24, 0), (64, 0), (100, 0),
                                     (128, 0), (128, 1), (256, 1), (128, 2), (256, 2), (384, 2)])
@pytest.mark.parametrize("beta,J", [(0.0, 1.0), (workloads.BETA_CRIT_CONFIG, 1.0), (0.3, -1.0),
                                    (3.0, 1.0), (300.0, 1.0)])
def test_heatbath_kernel_logic(emu, orc, L, rows5, beta, J):
    """The heat-bath word decision (five classes) against the oracle's heat-bath sweeps:
    per-word loop, row kernel, and the queued kernel's lock-step then per-lane blocks."""
    seed, stream, n, ctr = 55 + L, 3, 3, 4
    ref = orc.init(L, seed, stream)
    W = (L * L // 2 + 63) // 64
    words = np.ascontiguousarray(pack(ref).reshape(-1))
    T = np.ascontiguousarray(orc.thresholds(beta, J, "heatbath"), dtype=np.uint64)
    for s in range(n):
        for c in (0, 1):
            emu.emu_half_sweep5(_p(words), L, c, _p(T), 2 * (ctr + s) + c, seed, stream, rows5)
    orc.sweeps(ref, beta, J, seed, stream, n, ctr, rule="heatbath")
    assert np.array_equal(words.reshape(2, W), pack(ref))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_lane_pair_block_decisions_equal_plane_by_plane(emu, seed):
    """A lane pair evaluates two consecutive blocks at once: each reduced to
    the spins it decides and flips on its own, then applied in order.  That
    must leave exactly the state that applying the four planes in order
    leaves, for any pending set, classes and thresholds."""
    assert emu.emu_block_decision_check(seed, 20000) == 0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_plain_start_state_equals_the_class_split(emu, seed):
    """The queued row kernel's plain start state (flipped word, pending and
    class-A masks straight from the pair-level terms, without the "two or
    more" mask) equals the class split followed by the general start, for
    random words and both signs of J."""
    assert emu.emu_start_plain_check(seed, 20000) == 0


@pytest.mark.parametrize("L", [128, 256, 384, 512, 640])
def test_batch_row_aligned_neighbours_equal_the_general_extraction(emu, L):
    """For L % 128 == 0 the batch kernel reads whole words for the vertical
    neighbours and one edge word for the side neighbour; that must equal the
    general funnel-shift extraction for every word of both colours."""
    assert emu.emu_aligned_neighbours_check(L, L + 1) == 0
    assert emu.emu_aligned_row_check() == 0


@pytest.mark.parametrize("L", [64, 128, 192, 320, 448, 576, 704])
def test_batch_half_aligned_neighbours_equal_the_general_extraction(emu, L):
    """For L % 64 == 0 a colour row is a whole number of 32-bit halves: the
    vertical neighbours are whole halves H/32 away and the side neighbour one
    edge half; that must equal the general funnel-shift extraction for every
    word of both colours (sizes with an odd number of halves per row, whose
    words straddle rows, and whole-word rows alike)."""
    assert emu.emu_half_aligned_neighbours_check(L, L + 3) == 0
    assert emu.emu_half_row_check() == 0


@pytest.mark.parametrize("L", [4, 6, 10, 14, 16, 24, 30, 48, 50, 96, 100, 126, 130, 200, 300, 722])
def test_batch_general_neighbours_32bit_equal_the_64bit_extraction(emu, L):
    """The batch kernel's general extraction on 32-bit halves (funnel shifts of
    three halves, 32-bit wrapped positions) equals the 64-bit extraction for
    every word of both colours, including the partial last word and the
    cyclic continuation."""
    assert emu.emu_ext32_neighbours_check(L, L + 11) == 0
