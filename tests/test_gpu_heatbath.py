"""Heat-bath rule (Sec. 2) on the GPU: bit-exact parity with the oracle's
heat-bath sweeps through the C ABI, for the general and the row-aligned
kernels, and run-splitting invariance."""
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


@pytest.mark.parametrize("L", [4, 10, 24, 64, 128, 256, 384, 1000, 1024, 8192])
@pytest.mark.parametrize("beta,J", [(0.0, 1.0), (workloads.BETA_CRIT_CONFIG, 1.0), (0.3, -1.0),
                                    (3.0, 1.0)])
def test_heatbath_parity(gpu, orc, L, beta, J):
    print(f"heat bath L={L} beta={beta} J={J}", flush=True)
    seed, stream, n, ctr = 900 + L, 2, (4 if L <= 1024 else 2), 5
    lat = gpu.Lattice(L, seed=seed, stream_id=stream)
    lat.sweep(beta, J, n, ctr, rule="heatbath")
    ref = orc.init(L, seed, stream)
    orc.sweeps(ref, beta, J, seed, stream, n, ctr, rule="heatbath")
    assert np.array_equal(lat.packed(), pack(ref))
    assert lat.observables() == orc.observables(ref)


def test_heatbath_16384_full_lattice(gpu, orc):
    L, seed = 16384, 44
    print("heat bath L=16384, 1 sweep", flush=True)
    lat = gpu.Lattice(L, seed=seed)
    lat.sweep(0.44, 1.0, 1, 0, rule="heatbath")
    ref = orc.init(L, seed, 0)
    orc.sweeps(ref, 0.44, 1.0, seed, 0, 1, 0, rule="heatbath")
    assert np.array_equal(lat.packed(), pack(ref))


@pytest.mark.parametrize("L", [96, 256])
def test_heatbath_split_invariance(gpu, L):
    a = gpu.Lattice(L, seed=3)
    b = gpu.Lattice(L, seed=3)
    a.sweep(0.41, 1.0, 7, 0, rule="heatbath")
    b.sweep(0.41, 1.0, 3, 0, rule="heatbath")
    b.sweep(0.41, 1.0, 4, 3, rule="heatbath")
    assert np.array_equal(a.packed(), b.packed())
