"""The batched sweep without allocation (ising_batch_sweep_noalloc) against
the batch handle's sweep: identical lattices bit for bit, on two calls in a
row, the second on fewer lattices; sizes beyond its fixed array rejected."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def gpu():
    import torch

    import paper_1906_06297_amd as m

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m.load()
    return m


def handle_result(gpu, Ls, betas, seeds, streams, start, nsweeps, counter):
    b = gpu.Batch(Ls, betas, 1.0, seeds, streams)
    b.words.copy_(start)
    b.set_counter(counter)
    b.sweep(nsweeps)
    out = b.words.clone()
    b.close()
    return out


def test_noalloc_sweep_equals_the_batch_handle(gpu):
    import torch

    Ls, betas, seeds, streams = workloads.batched_lattices()
    n1 = 700  # the first 700 lattices of the batched workload
    Ls1, betas1 = [int(v) for v in Ls[:n1]], [float(v) for v in betas[:n1]]
    seeds1 = [int(v) for v in seeds[:n1]]
    streams1 = [int(v) for v in streams[:n1]]
    init = gpu.Batch(Ls1, betas1, 1.0, seeds1, streams1)
    init.init()
    start = init.words.clone()
    init.close()
    for call, (n, nsweeps, counter) in enumerate(((n1, 40, 5), (230, 17, 123456789012))):
        say(f"no-alloc call {call + 1}: {n} lattices, {nsweeps} sweeps from counter {counter}")
        Ls_c, betas_c, seeds_c, streams_c = Ls1[:n], betas1[:n], seeds1[:n], streams1[:n]
        words_c = int(gpu.batch_words(Ls_c))
        start_c = start[:words_c].contiguous()
        want = handle_result(gpu, Ls_c, betas_c, seeds_c, streams_c, start_c, nsweeps, counter)
        got = start_c.clone()
        gpu.batch_sweep_noalloc(Ls_c, betas_c, 1.0, seeds_c, streams_c, got, nsweeps, counter)
        torch.cuda.synchronize()
        assert not torch.equal(got, start_c)
        assert torch.equal(got, want)


def test_noalloc_rejects_more_lattices_than_its_array(gpu):
    import torch

    n = 4097
    Ls = [4] * n
    words = torch.zeros(int(gpu.batch_words(Ls)), dtype=torch.int64, device="cuda")
    with pytest.raises(gpu.IsingError) as e:
        gpu.batch_sweep_noalloc(Ls, [0.4] * n, 1.0, [1] * n, list(range(n)), words, 1, 0)
    assert e.value.code == -2
