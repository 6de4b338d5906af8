"""The largest lattices the library accepts (L * L / 128 just below 2^32 words
per colour, 64 GiB of spins): every 32-bit word index and counter word at its
limit.  After two sweeps, sampled 64 x 64 blocks (with the periodic seams)
agree with the oracle's windowed evolution, whose inner sites are exact."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def spins_at(words, L, rows, cols):
    """Spins (+1/-1) at the grid rows x cols, gathered from the packed device words."""
    import torch

    H, W = L // 2, (L * L // 2 + 63) // 64
    ii, jj = np.meshgrid(rows, cols, indexing="ij")
    c = (ii + jj) & 1
    n = ii.astype(np.int64) * H + (jj >> 1)
    widx = torch.as_tensor((c * W + (n >> 6)).reshape(-1), device=words.device)
    w = words[widx].cpu().numpy().view(np.uint64).reshape(ii.shape)
    bits = (w >> (n & 63).astype(np.uint64)) & np.uint64(1)
    return np.where(bits == 1, 1, -1).astype(np.int8)


@pytest.mark.parametrize("L", [741376, 741454])  # largest row-aligned, largest overall
def test_largest_lattice_sampled_windows(gpu_max, orc, L):
    import torch

    m = gpu_max
    beta, seed, stream, n = workloads.BETA_CRIT_CONFIG, 5, 1, 2
    print(f"L={L}: init + {n} sweeps", flush=True)
    lat = m.Lattice(L, seed=seed, stream_id=stream)
    lat.sweep(beta, 1.0, n, 0)
    torch.cuda.synchronize()
    margin, blk = 2 * n + 1, 64
    rng = np.random.default_rng(L)
    corners = [(0, 0), (L - 32, L - 32), (L - 1, 7)] + [tuple(int(v) for v in rng.integers(0, L, 2))
                                                       for _ in range(3)]
    for ci, cj in corners:
        i0, j0 = ci - margin, cj - margin
        win = orc.window_init(L, i0, j0, blk + 2 * margin, blk + 2 * margin, seed, stream)
        orc.window_sweeps(win, L, i0, j0, beta, 1.0, seed, stream, n, 0)
        inner = win[margin:margin + blk, margin:margin + blk]
        got = spins_at(lat.words, L, (np.arange(blk) + ci) % L, (np.arange(blk) + cj) % L)
        assert np.array_equal(got, inner), f"window at {(ci, cj)} differs"
    del lat
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def gpu_max():
    import torch

    import paper_1906_06297_amd as m

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m.load()
    free, _ = torch.cuda.mem_get_info()
    if free < 72 * (1 << 30):
        pytest.skip("needs 72 GiB of free device memory")
    return m
