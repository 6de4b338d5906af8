"""Bit-exact parity of the HIP path (through the C ABI) with the CPU oracle.

Every comparison is on the packed words or the int8 lattice, bit for bit, or
on exact int64 observables."""
import numpy as np
import pytest

import workloads
from layout import pack, unpack

pytestmark = pytest.mark.gpu

SIZES = [4, 6, 8, 10, 12, 16, 24, 30, 48, 64, 96, 128, 192, 256, 384, 640, 1000, 1024]


@pytest.fixture(scope="module")
def gpu():
    import torch

    import paper_1906_06297_amd as m

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m.load()
    return m


def _sync():
    import torch

    torch.cuda.synchronize()


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("L", SIZES)
def test_init_parity(gpu, orc, L):
    say(f"init parity L={L}")
    lat = gpu.Lattice(L, seed=5 + L, stream_id=3)
    assert np.array_equal(lat.packed(), pack(orc.init(L, 5 + L, 3)))


@pytest.mark.parametrize("L", SIZES)
@pytest.mark.parametrize("beta,J", [(0.0, 1.0), (0.30, 1.0), (workloads.BETA_CRIT_CONFIG, 1.0),
                                    (0.5, 1.0), (8.0, 1.0), (0.35, -1.0), (0.6, 0.0)])
def test_sweep_parity(gpu, orc, L, beta, J):
    say(f"sweep parity L={L} beta={beta} J={J}")
    seed, stream, n, ctr = 1000 + L, 7, 6, 11
    lat = gpu.Lattice(L, seed=seed, stream_id=stream)
    lat.sweep(beta, J, n, ctr)
    ref = orc.init(L, seed, stream)
    orc.sweeps(ref, beta, J, seed, stream, n, ctr)
    got = lat.packed()
    assert np.array_equal(got, pack(ref)), f"first mismatch {np.argwhere(got != pack(ref))[:4]}"


@pytest.mark.parametrize("L", [4, 10, 24, 64, 128, 256, 384, 1000])
def test_set_get_roundtrip_and_observables(gpu, orc, L):
    say(f"set/get/observables L={L}")
    lat = gpu.Lattice(L, seed=1)
    for p_up in (0.5, 0.9, 1.0, 0.0):
        s = workloads.random_spins(L, 31 * L, p_up)
        lat.set_spins(s)
        assert np.array_equal(lat.get_spins(), s)
        assert np.array_equal(lat.packed(), pack(s))
        assert lat.observables() == orc.observables(s)


def test_correctness_workload_trace(gpu, orc):
    """L=64, beta=0.4406868, seed 42, 1000 sweeps: every sweep's (E, M) and the
    final lattice agree exactly."""
    cfg = workloads.CORRECTNESS
    L, n = cfg["L"], cfg["nsweeps"]
    say("correctness workload L=64, 1000 sweeps")
    lat = gpu.Lattice(L, seed=cfg["seed"], stream_id=cfg["stream"])
    bond, mag = lat.sweep_traced(cfg["beta"], cfg["J"], n, cfg["rng_counter"])
    ref = orc.init(L, cfg["seed"], cfg["stream"])
    rb, rm = orc.sweeps(ref, cfg["beta"], cfg["J"], cfg["seed"], cfg["stream"], n,
                        cfg["rng_counter"], trace=True)
    assert np.array_equal(bond.cpu().numpy(), rb)
    assert np.array_equal(mag.cpu().numpy(), rm)
    assert np.array_equal(lat.get_spins(), ref)


@pytest.mark.parametrize("L", [24, 64, 256])
def test_split_invariance(gpu, L):
    """Sweeps split across calls with consecutive counters give the same lattice."""
    say(f"split invariance L={L}")
    a = gpu.Lattice(L, seed=9)
    a.sweep(0.44, 1.0, 7, 3)
    b = gpu.Lattice(L, seed=9)
    b.sweep(0.44, 1.0, 2, 3)
    b.sweep(0.44, 1.0, 5, 5)
    assert np.array_equal(a.packed(), b.packed())


def test_zero_sweeps_is_a_no_op(gpu):
    lat = gpu.Lattice(64, seed=2)
    before = lat.packed().copy()
    lat.sweep(0.44, 1.0, 0, 0)
    assert np.array_equal(lat.packed(), before)


def test_padding_bits_stay_zero(gpu):
    L = 24  # 288 spins per colour: the last word holds 32 spins
    lat = gpu.Lattice(L, seed=4)
    lat.sweep(0.0, 1.0, 3, 0)  # beta = 0 flips every spin
    w = lat.packed()
    assert (int(w[0, -1]) >> 32) == 0 and (int(w[1, -1]) >> 32) == 0


def test_row_aligned_4096_full(gpu, orc):
    """The headline kernel on fewer tiles for the headline's full 200 sweeps."""
    L, seed, n = 4096, 21, workloads.HEADLINE["nsweeps"]
    say(f"full-lattice parity L=4096, {n} sweeps")
    lat = gpu.Lattice(L, seed=seed)
    lat.sweep(workloads.BETA_CRIT_CONFIG, 1.0, n, 0)
    ref = orc.init(L, seed, 0)
    orc.sweeps(ref, workloads.BETA_CRIT_CONFIG, 1.0, seed, 0, n, 0)
    assert np.array_equal(lat.packed(), pack(ref))
    assert lat.observables() == orc.observables(ref)


def test_headline_full_lattice_first_sweeps(gpu, orc):
    """L = 65536 in the benchmark's launch configuration: the whole lattice
    (2^32 spins) bit for bit after the first 4 sweeps at beta_c."""
    from layout import pack_rows

    cfg = workloads.HEADLINE
    L, n, beta = cfg["L"], 4, workloads.BETA_CRIT_CONFIG
    say("headline size, whole lattice, 4 sweeps")
    lat = gpu.Lattice(L, seed=cfg["seed"], stream_id=cfg["stream"])
    lat.sweep(beta, cfg["J"], n, 0)
    got = lat.packed()
    say("oracle: 4 sweeps at L = 65536")
    ref = orc.init(L, cfg["seed"], cfg["stream"])
    orc.sweeps(ref, beta, cfg["J"], cfg["seed"], cfg["stream"], n, 0)
    assert np.array_equal(got, pack_rows(ref))


@pytest.mark.parametrize("beta", workloads.HEADLINE["betas"])
def test_headline_size_sampled_windows(gpu, orc, beta):
    """L = 65536 in the benchmark's launch configuration: after 3 sweeps from the
    seed-7 start, sampled 96x96 blocks (including the periodic seams) agree with
    the oracle's windowed evolution, whose inner sites are exact."""
    cfg = workloads.HEADLINE
    L, n = cfg["L"], 3
    say(f"headline-size windows beta={beta}")
    lat = gpu.Lattice(L, seed=cfg["seed"], stream_id=cfg["stream"])
    lat.sweep(beta, cfg["J"], n, 0)
    _sync()
    Wr = L // 128  # words per colour row (row-aligned size)
    rows_all = lat.words.view(2, L, Wr)
    margin = 2 * n + 1
    blk = 96
    rng = np.random.default_rng(17)
    corners = [(0, 0), (L - 48, L - 48), (L // 2, 0)] + [tuple(int(v) for v in rng.integers(0, L, 2)) for _ in range(5)]
    for (ci, cj) in corners:
        i0, j0 = ci - margin, cj - margin
        win = orc.window_init(L, i0, j0, blk + 2 * margin, blk + 2 * margin, cfg["seed"], cfg["stream"])
        orc.window_sweeps(win, L, i0, j0, beta, cfg["J"], cfg["seed"], cfg["stream"], n, 0)
        inner = win[margin:margin + blk, margin:margin + blk]
        rows = (np.arange(blk) + ci) % L
        cols = (np.arange(blk) + cj) % L
        import torch
        rw = rows_all[:, torch.as_tensor(rows, device=lat.words.device), :].cpu().numpy().view(np.uint64)
        ii, jj = np.meshgrid(rows, cols, indexing="ij")
        c = (ii + jj) & 1
        jc = jj >> 1
        a_idx = np.broadcast_to(np.arange(blk)[:, None], (blk, blk))
        word = rw[c, a_idx, jc >> 6]
        bits = (word >> (jc & 63).astype(np.uint64)) & np.uint64(1)
        got = np.where(bits == 1, 1, -1).astype(np.int8)
        assert np.array_equal(got, inner), f"window at {(ci, cj)} differs"


@pytest.mark.parametrize("variant", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("L,nsw", [(128, 6), (384, 6), (1000, 4), (1024, 4), (8190, 2), (8192, 2),
                                   (8320, 2), (16384, 1)])
@pytest.mark.parametrize("beta,J", [(workloads.BETA_CRIT_CONFIG, 1.0), (0.40, 1.0), (0.5, 1.0),
                                    (0.33, -1.0), (0.0, 1.0), (6.0, 1.0)])
def test_every_kernel_variant_bit_exact(gpu, orc, variant, L, nsw, beta, J):
    """Default (by size), general-geometry kernel, the row kernel without the
    queue and the queued row kernel with 32-, 16- and 8-row bands at every size
    give the oracle's lattice.  Sizes include rows that straddle words (1000,
    8190: every choice takes the general kernel), wavefronts with idle lanes (384: 3 words per colour row; 8320: 65)
    and rows of whole 64-word segments (8192: one wavefront per row, 16384:
    two)."""
    say(f"variant {variant} L={L} beta={beta} J={J}")
    seed, stream = 300 + L, 1
    gpu.set_sweep_kernel(variant)
    try:
        lat = gpu.Lattice(L, seed=seed, stream_id=stream)
        lat.sweep(beta, J, nsw, 2)
        got = lat.packed()
    finally:
        gpu.set_sweep_kernel(0)
    key = (L, nsw, beta, J, seed, stream)
    ref = _ref_cache.get(key)
    if ref is None:
        s = orc.init(L, seed, stream)
        orc.sweeps(s, beta, J, seed, stream, nsw, 2)
        ref = _ref_cache[key] = pack(s)
    assert np.array_equal(got, ref)


_ref_cache = {}
