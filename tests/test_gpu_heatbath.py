"""Heat-bath rule (Sec. 2) on the GPU: bit-exact parity with the oracle's
heat-bath sweeps through the C ABI, for every kernel choice (default by size,
general, row kernel without queue, queued with 32-, 16-, 8-row bands), and
run-splitting invariance."""
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


# 128, 384: fewer than 64 words per row; 8192: one 64-word segment per row;
# 8320: 65 words per row, a partial last segment; 16384: two segments
@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("L,n", [(128, 4), (384, 4), (1024, 3), (8192, 2), (8320, 2), (16384, 1)])
@pytest.mark.parametrize("beta,J", [(workloads.BETA_CRIT_CONFIG, 1.0), (0.3, -1.0), (3.0, 1.0)])
def test_heatbath_every_kernel(gpu, orc, variant, L, n, beta, J):
    print(f"heat bath variant={variant} L={L} beta={beta} J={J}", flush=True)
    seed, stream, ctr = 70 + L, 1, 3
    lat = gpu.Lattice(L, seed=seed, stream_id=stream)
    gpu.set_sweep_kernel(variant)
    try:
        lat.sweep(beta, J, n, ctr, rule="heatbath")
    finally:
        gpu.set_sweep_kernel(0)
    key = (L, n, beta, J)
    ref = _ref5.get(key)
    if ref is None:
        ref = orc.init(L, seed, stream)
        orc.sweeps(ref, beta, J, seed, stream, n, ctr, rule="heatbath")
        _ref5[key] = ref
    assert np.array_equal(lat.packed(), pack(ref))


_ref5 = {}


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


def test_heatbath_headline_size_full_lattice(gpu, orc):
    """L = 65536 with the default kernel there (queued, 16-row bands): the whole
    lattice bit for bit after one heat-bath sweep at beta_c."""
    from layout import pack_rows

    cfg = workloads.HEADLINE
    L, beta = cfg["L"], workloads.BETA_CRIT_CONFIG
    print("heat bath L=65536, 1 sweep", flush=True)
    lat = gpu.Lattice(L, seed=cfg["seed"], stream_id=cfg["stream"])
    lat.sweep(beta, cfg["J"], 1, 0, rule="heatbath")
    got = lat.packed()
    del lat
    ref = orc.init(L, cfg["seed"], cfg["stream"])
    orc.sweeps(ref, beta, cfg["J"], cfg["seed"], cfg["stream"], 1, 0, rule="heatbath")
    assert np.array_equal(got, pack_rows(ref))
