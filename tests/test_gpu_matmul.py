"""The matrix-multiply formulation (fp16 MFMA neighbour sums) on the GPU
through the C ABI: layout round trip, bit-exact sweeps against the oracle in
both the fused and the three-kernel form, agreement with the bit-packed
sweep at the headline size, and argument checks."""
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


def say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("L", [256, 512, 768])
def test_layout_round_trip(gpu, L):
    say(f"matmul round trip L={L}")
    a = gpu.Lattice(L, seed=3 + L, stream_id=1)
    before = a.packed().copy()
    mm = gpu.MatmulLattice(a)
    b = gpu.Lattice(L, seed=0)
    mm.to_lattice(b)
    assert np.array_equal(b.packed(), before)


# 256: one sub-lattice (every edge term wraps onto the same sub-lattice);
# 512, 768: 2 x 2 and 3 x 3 sub-lattices.
@pytest.mark.parametrize("fused", [True, False])
@pytest.mark.parametrize("L", [256, 512, 768])
@pytest.mark.parametrize("beta,J", [(0.44, 1.0), (1.2, 1.0), (0.5, -1.0), (0.0, 1.0), (9.0, 1.0),
                                    (0.3, -1.0)])
def test_matmul_sweep_matches_oracle(gpu, orc, fused, L, beta, J):
    say(f"matmul fused={fused} L={L} beta={beta} J={J}")
    seed, stream, n, ctr = 40 + L, 2, 3, 7
    lat = gpu.Lattice(L, seed=seed, stream_id=stream)
    mm = gpu.MatmulLattice(lat, fused=fused)
    mm.sweep(beta, J, n, ctr)
    mm.to_lattice(lat)
    ref = orc.init(L, seed, stream)
    orc.sweeps(ref, beta, J, seed, stream, n, ctr)
    assert np.array_equal(lat.packed(), pack(ref))


@pytest.mark.parametrize("fused", [True, False])
def test_matmul_sweep_matches_oracle_16384(gpu, orc, fused):
    """64 x 64 sub-lattices, two sweeps at beta_c."""
    L, seed, stream, n, ctr, beta = 16384, 5, 0, 2, 1, 0.4406868
    say(f"matmul fused={fused} L={L}")
    lat = gpu.Lattice(L, seed=seed, stream_id=stream)
    mm = gpu.MatmulLattice(lat, fused=fused)
    mm.sweep(beta, 1.0, n, ctr)
    mm.to_lattice(lat)
    ref = orc.init(L, seed, stream)
    orc.sweeps(ref, beta, 1.0, seed, stream, n, ctr)
    assert np.array_equal(lat.packed(), pack(ref))


def test_matmul_equals_bitpacked_at_65536(gpu):
    """The headline lattice (seed 7, beta_c): one sweep of each matmul form
    equals one sweep of the bit-packed kernel, whose full-size agreement with
    the oracle the parity tests establish."""
    import torch

    L, beta = 65536, 0.4406868
    say("matmul vs bit-packed L=65536")
    ref = gpu.Lattice(L, seed=7)
    ref.sweep(beta, 1.0, 1, 0)
    want = ref.words.clone()
    del ref
    for fused in (True, False):
        lat = gpu.Lattice(L, seed=7)
        mm = gpu.MatmulLattice(lat, fused=fused)
        mm.sweep(beta, 1.0, 1, 0)
        mm.to_lattice(lat)
        assert torch.equal(lat.words, want), f"fused={fused}"
        del mm, lat
        torch.cuda.empty_cache()


def test_matmul_argument_checks(gpu):
    from paper_1906_06297_amd import IsingError

    lib = gpu.load()
    assert lib.ising_mm_lattice_bytes(384) == -1
    assert lib.ising_mm_lattice_bytes(512) == 2 * 512 * 512
    assert lib.ising_mm_sums_bytes(512) == 512 * 512
    with pytest.raises(ValueError):
        gpu.MatmulLattice(gpu.Lattice(384, seed=1))
    mm = gpu.MatmulLattice(gpu.Lattice(256, seed=1), fused=False)
    mm.sums = mm.sums[: 8]  # too small
    with pytest.raises(IsingError):
        mm.sweep(0.4, 1.0, 1, 0)
