"""+-J spin glass on the GPU through the C ABI: the bond generator against the
oracle's, bit-exact sweeps and exact observables against the oracle, the
ferromagnetic and gauge reductions, and argument checks."""
import numpy as np
import pytest

from layout import pack

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    import paper_1906_06297_amd as m

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m.load()
    return m


def unpack_bonds(words, L):
    """Device bond arrays -> (Jr, Jd) int8 +1/-1 (host side, independent of the library)."""
    W = (L * L // 2 + 63) // 64
    w = words.cpu().numpy().view(np.uint64).reshape(W, 4).T  # word k of array x at 4 k + x
    H = L // 2
    Jr = np.zeros((L, L), np.int8)
    Jd = np.zeros((L, L), np.int8)
    for x in range(4):
        c = x & 1
        bits = ((w[x][:, None] >> np.arange(64, dtype=np.uint64)[None, :]) & np.uint64(1)).reshape(-1)
        n = np.arange(L * H)
        i, jc = n // H, n % H
        j = 2 * jc + ((i + c) & 1)
        (Jr if x < 2 else Jd)[i, j] = np.where(bits[: L * H] == 1, -1, 1)
    return Jr, Jd


@pytest.mark.parametrize("L", [128, 384, 1024])
def test_bond_generator_matches_oracle(gpu, orc, L):
    b = gpu.GlassBonds(L, seed=11, stream_id=3)
    Jr, Jd = orc.glass_couplings(L, 11, 3)
    got = unpack_bonds(b.words, L)
    assert np.array_equal(got[0], Jr) and np.array_equal(got[1], Jd)


# 128 and 384: fewer than 64 words per row (no cross-lane side shift in the
# queued kernel); 8192: 64 words per row; 16384 with 3 sweeps: several wave
# segments per row and bands that end mid-lattice.
@pytest.mark.parametrize("variant", [0, 2, 3, 4, 5])
@pytest.mark.parametrize("L", [128, 256, 384, 1024, 8192])
@pytest.mark.parametrize("beta,J", [(0.44, 1.0), (1.2, 1.0), (0.5, -1.0), (0.0, 1.0), (9.0, 1.0)])
def test_glass_parity(gpu, orc, variant, L, beta, J):
    print(f"glass variant={variant} L={L} beta={beta} J={J}", flush=True)
    seed, stream, n, ctr = 70 + L, 1, (3 if L <= 1024 else 1), 2
    bonds = gpu.GlassBonds(L, seed=5 + L, stream_id=0)
    lat = gpu.Lattice(L, seed=seed, stream_id=stream)
    gpu.set_sweep_kernel(variant)
    try:
        lat.glass_sweep(bonds, beta, J, n, ctr)
    finally:
        gpu.set_sweep_kernel(0)
    Jr, Jd = orc.glass_couplings(L, 5 + L, 0)
    ref = orc.init(L, seed, stream)
    orc.glass_sweeps(ref, Jr, Jd, beta, J, seed, stream, n, ctr)
    assert np.array_equal(lat.packed(), pack(ref))
    assert lat.glass_observables(bonds) == orc.glass_observables(ref, Jr, Jd)


@pytest.mark.parametrize("L,n", [(16384, 2), (8320, 2)])
def test_glass_parity_large(gpu, orc, L, n):
    """Several 64-word wave segments per row (16384), a row length that is not
    a multiple of 64 words with a partial last segment (8320 = 65 words)."""
    print(f"glass large L={L}", flush=True)
    seed, stream, ctr, beta, J = 3, 2, 5, 0.44, 1.0
    bonds = gpu.GlassBonds(L, seed=9, stream_id=1)
    lat = gpu.Lattice(L, seed=seed, stream_id=stream)
    lat.glass_sweep(bonds, beta, J, n, ctr)
    Jr, Jd = orc.glass_couplings(L, 9, 1)
    ref = orc.init(L, seed, stream)
    orc.glass_sweeps(ref, Jr, Jd, beta, J, seed, stream, n, ctr)
    assert np.array_equal(lat.packed(), pack(ref))


def test_ferromagnetic_bonds_give_the_plain_sweep(gpu):
    L = 256
    one = np.ones((L, L), np.int8)
    bonds = gpu.GlassBonds(L, right=one, down=one)
    a = gpu.Lattice(L, seed=9)
    b = gpu.Lattice(L, seed=9)
    a.glass_sweep(bonds, 0.43, 1.0, 5, 0)
    b.sweep(0.43, 1.0, 5, 0)
    assert np.array_equal(a.packed(), b.packed())
    assert a.glass_observables(bonds) == b.observables()


def test_gauge_transform_on_the_gpu(gpu, orc):
    L = 128
    rng = np.random.default_rng(4)
    Jr, Jd = orc.glass_couplings(L, 8, 0)
    tau = np.where(rng.random((L, L)) < 0.5, -1, 1).astype(np.int8)
    a = gpu.Lattice(L, seed=2)
    s0 = a.get_spins()
    a.glass_sweep(gpu.GlassBonds(L, right=Jr, down=Jd), 0.6, 1.0, 4, 0)
    b = gpu.Lattice(L, seed=2)
    b.set_spins((tau * s0).astype(np.int8))
    Jr2 = (tau * Jr * np.roll(tau, -1, 1)).astype(np.int8)
    Jd2 = (tau * Jd * np.roll(tau, -1, 0)).astype(np.int8)
    b.glass_sweep(gpu.GlassBonds(L, right=Jr2, down=Jd2), 0.6, 1.0, 4, 0)
    assert np.array_equal(b.get_spins(), tau * a.get_spins())


def test_glass_argument_checks(gpu):
    from paper_1906_06297_amd import IsingError

    with pytest.raises(IsingError):
        gpu.GlassBonds(100, seed=1)  # rows of whole words only
    lat = gpu.Lattice(256, seed=1)
    small = gpu.GlassBonds(128, seed=1)
    with pytest.raises(IsingError):
        lat.glass_sweep(small, 0.4, 1.0, 1, 0)  # bond array too small for L = 256


def test_glass_headline_size_full_lattice(gpu, orc):
    """The glass workload at L = 65536 with the default kernel (queued, 8-row
    bands): the whole lattice bit for bit after one sweep."""
    import workloads
    from layout import pack_rows

    cfg = workloads.GLASS
    L, beta = cfg["L"], cfg["betas"][1]
    print("glass L=65536, 1 sweep", flush=True)
    bonds = gpu.GlassBonds(L, seed=cfg["coupling_seed"], stream_id=0)
    lat = gpu.Lattice(L, seed=cfg["seed"], stream_id=cfg["stream"])
    lat.glass_sweep(bonds, beta, cfg["J"], 1, 0)
    got = lat.packed()
    del lat, bonds
    Jr, Jd = orc.glass_couplings(L, cfg["coupling_seed"], 0)
    ref = orc.init(L, cfg["seed"], cfg["stream"])
    orc.glass_sweeps(ref, Jr, Jd, beta, cfg["J"], cfg["seed"], cfg["stream"], 1, 0)
    assert np.array_equal(got, pack_rows(ref))
