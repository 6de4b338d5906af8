"""The learned proposal on the GPU (through the C ABI) against the oracle:
log-probabilities, gradients, bit-identity of the sampler's and the
evaluator's probabilities, sampling frequencies, an exact Metropolis-Hastings
chain, training, and the batch <-> int8 conversions."""
import numpy as np
import pytest

import workloads
from layout import pack
from oracle import arnet as ref, exact, stats

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    import paper_1906_06297_amd as m

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    m.load()
    return m


def say(*a):
    print(*a, flush=True)


def spins_t(x):
    import torch

    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.int8)).cuda()


def rand_spins(B, L, seed, p_up=0.5):
    return np.where(np.random.default_rng(seed).random((B, L, L)) < p_up, 1, -1).astype(np.int8)


@pytest.mark.parametrize("C", [32, 64])
@pytest.mark.parametrize("L", [4, 6, 8, 16])
def test_log_prob_matches_oracle(gpu, C, L):
    say(f"log_prob C={C} L={L}")
    th = ref.init_params(C, 100 + L, scale=1.2)
    net = gpu.ARNet(L, C, 64)
    net.set_params(th.astype(np.float32))
    x = rand_spins(13, L, L, 0.7)
    logq, logits = net.log_prob(spins_t(x), logits=True)
    want_logit, _ = ref.forward(x, th, C, emulate_bf16=True)
    diff = np.abs(logits.cpu().numpy() - want_logit)
    # float32 (GPU) and double (oracle) sums can round an activation to
    # neighbouring bf16 values; that moves a few logits by ~1e-3 relative
    assert diff.mean() < 1e-3 and np.all(diff <= 0.02 + 0.01 * np.abs(want_logit))
    want = ref.log_q_exact(x, th, C, emulate_bf16=True)
    got = logq.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - want) <= 1e-3 * np.abs(want) + 1e-4), (got, want)
    # and against the unrounded float model: the bf16 network stays within 1e-3 relative
    smooth = ref.log_q(x, th, C)
    assert np.all(np.abs(got - smooth) <= 1e-2 * np.abs(smooth) + 0.05)
    net.close()


@pytest.mark.parametrize("C", [32, 64])
def test_gradient_matches_oracle(gpu, C):
    L, B = 8, 12
    say(f"gradient C={C}")
    th = ref.init_params(C, 5, scale=1.0) + np.random.default_rng(6).normal(0, 0.05, ref.num_params(C))
    net = gpu.ARNet(L, C, 32)
    net.set_params(th.astype(np.float32))
    x = rand_spins(B, L, 7)
    loss, g = net.gradient(spins_t(x))
    nll, want = ref.nll_and_grad(x, th, C, emulate_bf16=True)
    assert abs(float(loss.item()) - nll) <= 1e-4 * abs(nll)
    got = g.cpu().numpy().astype(np.float64)
    # per parameter block: relative error of the block vector
    p_got, p_want = ref.unflatten(got, C), ref.unflatten(want, C)
    for k in p_want:
        a, b = np.atleast_1d(p_got[k]).ravel(), np.atleast_1d(p_want[k]).ravel()
        err = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-12)
        assert err < 2e-2, (k, err)
    net.close()


@pytest.mark.parametrize("C,L", [(32, 8), (64, 6), (32, 16)])
def test_sampler_matches_evaluator_bit_for_bit(gpu, C, L):
    say(f"sampler/evaluator C={C} L={L}")
    th = ref.init_params(C, 40 + L, scale=1.5)
    net = gpu.ARNet(L, C, 64)
    net.set_params(th.astype(np.float32))
    x, lq = net.sample(37, seed=11, stream_base=5, round=3)  # 37: a partial tile of 16
    lq2 = net.log_prob(x)
    assert np.array_equal(lq.cpu().numpy(), lq2.cpu().numpy())
    xs = x.cpu().numpy()
    assert set(np.unique(xs)) <= {-1, 1}
    want = ref.log_q_exact(xs, th, C, emulate_bf16=True)
    assert np.allclose(lq.cpu().numpy(), want, rtol=1e-3, atol=1e-4)
    # different rounds and streams give different samples; the same give the same
    x_same, _ = net.sample(37, seed=11, stream_base=5, round=3)
    x_other, _ = net.sample(37, seed=11, stream_base=5, round=4)
    assert np.array_equal(x_same.cpu().numpy(), xs)
    assert not np.array_equal(x_other.cpu().numpy(), xs)
    net.close()


def test_sampling_frequencies_match_q(gpu):
    C, L, n = 32, 2, 1 << 16
    th = ref.init_params(C, 77, scale=2.0)
    net = gpu.ARNet(L, C, n)
    net.set_params(th.astype(np.float32))
    x, lq = net.sample(n, seed=3)
    xs = x.cpu().numpy().reshape(n, -1)
    codes = ((xs > 0) * (1 << np.arange(L * L))).sum(axis=1)
    states = exact.all_states(L).astype(np.float64)
    q = np.exp(ref.log_q_exact(states, th, C, emulate_bf16=True))
    assert abs(q.sum() - 1) < 1e-9
    counts = np.bincount(codes, minlength=16)
    sd = np.sqrt(n * q * (1 - q))
    assert np.all(np.abs(counts - n * q) <= 5 * sd + 2), (counts, n * q)
    net.close()


def test_independence_chain_exact_on_4x4(gpu):
    """Learned-proposal Metropolis-Hastings keeps the Boltzmann distribution:
    chains started from exact 4x4 Boltzmann samples stay there (random-weight
    q, pure global moves)."""
    import torch

    C, L, beta, chains, rounds = 32, 4, 0.3, 1024, 160
    th = ref.init_params(C, 91, scale=0.5)
    net = gpu.ARNet(L, C, chains)
    net.set_params(th.astype(np.float32))
    states = exact.all_states(L)
    pi = exact.boltzmann_weights(L, beta)
    start = states[np.random.default_rng(5).choice(len(states), chains, p=pi)]
    state = spins_t(start)
    lq = net.log_prob(state)
    bond, _ = gpu.spins_observables(state, L)
    betaJ = torch.full((chains,), beta, dtype=torch.float32, device="cuda")
    E = np.empty((rounds, chains))
    M2 = np.empty((rounds, chains))
    acc_total = 0
    for r in range(1, rounds + 1):
        prop, lqp = net.sample(chains, seed=1, stream_base=0, round=r)
        bp, _ = gpu.spins_observables(prop, L)
        acc = gpu.mh_independence(state, lq, bond, prop, lqp, bp, betaJ, seed=2, stream_base=0,
                                  round=r)
        acc_total += int(acc.sum().item())
        _, mag = gpu.spins_observables(state, L)
        E[r - 1] = -bond.cpu().numpy() / 16
        M2[r - 1] = (mag.cpu().numpy() / 16) ** 2
    ex = exact.enumerate_lattice(L, beta)
    say(f"acceptance {acc_total / (chains * rounds):.3f}")
    assert acc_total > 0.02 * chains * rounds
    # the chains' state log q stays consistent with the evaluator
    assert np.array_equal(lq.cpu().numpy(), net.log_prob(state).cpu().numpy())
    for s_, target in ((E, ex["E_per_site"]), (M2, ex["m2"])):
        per_chain = s_.mean(axis=0)  # independent chains
        se = per_chain.std(ddof=1) / np.sqrt(chains)
        assert abs(per_chain.mean() - target) < 4.5 * se, (per_chain.mean(), target, se)
    net.close()


def test_training_lowers_the_loss(gpu, orc):
    import torch

    C, L = 32, 8
    net = gpu.ARNet(L, C, 256)
    net.set_params(ref.init_params(C, 12, scale=0.5).astype(np.float32))
    # ordered-phase data from the oracle sampler: mostly aligned configurations
    data = np.stack([orc.init(L, 500 + k, 0) for k in range(256)])
    for k in range(256):
        orc.sweeps(data[k], 0.6, 1.0, 500 + k, 0, 60, 0)
    d = spins_t(data)
    first = float(net.gradient(d)[0].item())
    for step in range(150):
        loss = net.train_step(d, 3e-3)
    last = float(loss.item())
    say(f"training loss {first:.2f} -> {last:.2f}")
    assert last < 0.7 * first
    net.close()


def test_batch_spin_conversions(gpu, orc):
    Ls = [4, 6, 16, 24, 64]
    b = gpu.Batch(Ls, [0.4] * 5, 1.0, [2] * 5, [0, 1, 2, 3, 4])
    b.init()
    sp = b.spins().cpu().numpy()
    o = 0
    for q, L in enumerate(Ls):
        assert np.array_equal(sp[o:o + L * L].reshape(L, L), orc.init(L, 2, q))
        o += L * L
    rnd = np.concatenate([rand_spins(1, L, L).reshape(-1) for L in Ls])
    b.set_spins(spins_t(rnd))
    o = 0
    for q, L in enumerate(Ls):
        assert np.array_equal(b.lattice(q).packed(), pack(rnd[o:o + L * L].reshape(L, L)))
        o += L * L
    b.close()
