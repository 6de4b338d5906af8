"""The learned proposal on the GPU (through the C ABI) against the oracle.

Tolerances (derived from the arithmetic; the network's weights are drawn
bf16-representable, so the GPU network and the plain model have the same
weights and the comparisons measure the kernels' arithmetic alone):

* logits: the GPU stores the activations of layers 1..5 rounded to bfloat16
  (relative error <= u = 2^-9 each) and sums in float32 (<= K 2^-24 of the sum
  of absolute products, K <= 5C + 1 terms).  ReLU is 1-Lipschitz, so by
  induction |h_l(GPU) - h_l| <= l (u + K 2^-24) A_l and
  |z(GPU) - z| <= (5u + 6 K 2^-24) A_6 (x 1.05 for second-order terms), with
  A_l the absolute-value forward pass (``oracle.arnet.forward_abs``).
* log q~: within 1e-3 relative of the plain model's, the bar set for the
  learned part.
* gradients at given forward values (``ising_arnet_gradient_at``: the
  activations and logits are inputs, so the result is unique): the backward
  signal is float32 and enters the MFMA products as two bf16 halves
  (representation error <= 2^-18 per layer, <= 5 layers, < 2^-15 in all),
  dlogit is formed in float32 (a few roundings, < 2^-20 relative), and every
  sum is float32 with at most S = 64 cpb + nblk + 25 C terms in series (rows
  per workgroup, workgroups, the transposed convolution), so
  |g(GPU) - g| <= (2^-15 + S 2^-24) G^abs element by element, G^abs the
  backward pass with absolute values (``oracle.arnet.grad_abs_from``).
* gradients end to end (forward and backward on the GPU): the forward pass
  rounds each activation to bf16 and decides each ReLU mask from a float32
  sum, and a few of those decisions differ from the double oracle's (about 1
  in 500 at layer 5 on these networks); a changed decision moves a gradient
  element by at most the terms that pass through it.  At least 99 % of the
  elements meet the bound above and every element is within 2^-5 G^abs.
"""
import numpy as np
import pytest

from layout import pack
from oracle import arnet as ref, exact

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -9
U_F32 = 2.0 ** -24
SAMPLE_MARGIN = 2.0 ** -9


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


def mixed_configs(B, L, seed, orc=None, n_ising=0, beta=0.44):
    """Random configurations of varying magnetisation; the first n_ising are
    oracle Metropolis configurations at beta (300 sweeps from a random start)."""
    rng = np.random.default_rng(seed)
    p = rng.uniform(0.1, 0.9, (B, 1, 1))
    x = np.where(rng.random((B, L, L)) < p, 1, -1).astype(np.int8)
    for k in range(n_ising):
        s = orc.init(L, seed + k, 0)
        orc.sweeps(s, beta, 1.0, seed + k, 0, 300, 0)
        x[k] = s
    return x


def bf16_params(C, seed, scale):
    """Seeded He-style weights with small random biases, rounded to bf16."""
    p = ref.unflatten(ref.init_params(C, seed, scale=scale), C)
    rng = np.random.default_rng(seed + 1)
    for k in p:
        if k.startswith("b"):
            p[k] = rng.normal(0, 0.1, np.shape(p[k]))
    return ref.bf16(ref.flatten(p, C))


def logit_tol(x, th, C):
    K = 5 * C + 1
    return 1.05 * (5 * U_BF16 + 6 * K * U_F32) * ref.forward_abs(x, th, C)


def check_log_prob(gpu, L, C, B, th, x, sample_idx):
    net = gpu.ARNet(L, C, B)
    net.set_params(th.astype(np.float32))
    logq, logits = net.log_prob(spins_t(x), logits=True)
    got_z = logits.cpu().numpy()[sample_idx].astype(np.float64)
    got_q = logq.cpu().numpy()[sample_idx].astype(np.float64)
    xs = x[sample_idx]
    want_z, _ = ref.forward(xs, th, C)  # the plain model, double, unrounded activations
    tol = logit_tol(xs, th, C)
    err = np.abs(got_z - want_z)
    ratio = err / np.maximum(tol, 1e-300)
    say(f"  logits: max |dz| {err.max():.3g}, mean {err.mean():.3g}, max |dz|/bound "
        f"{ratio.max():.3g}")
    assert np.all(err <= tol), np.unravel_index(np.argmax(ratio), err.shape)
    emu_z, _ = ref.forward(xs, th, C, emulate_bf16=True)
    d_emu = np.abs(got_z - emu_z) / (1.0 + np.abs(emu_z))
    say(f"  against the bf16-storage oracle: quantiles 50/99/99.9/100 % of |dz|/(1+|z|) "
        f"{np.quantile(d_emu, [0.5, 0.99, 0.999, 1.0])}")
    want_q = ref.log_q_exact(xs, th, C, emulate_bf16=False)
    rel = np.abs(got_q - want_q) / np.abs(want_q)
    say(f"  log q~: max relative difference {rel.max():.3g}")
    assert np.all(np.isfinite(want_q)) and np.all(rel <= 1e-3), (got_q, want_q)
    net.close()


@pytest.mark.parametrize("C", [32, 64])
@pytest.mark.parametrize("L", [4, 6, 8, 16])
def test_log_prob_against_fp32_model(gpu, C, L):
    say(f"log_prob C={C} L={L}")
    th = bf16_params(C, 100 + L, scale=1.0)
    x = mixed_configs(13, L, L)
    check_log_prob(gpu, L, C, 13, th, x, np.arange(13))


@pytest.mark.parametrize("L,C,B,n_check", [(32, 32, 4096, 96), (64, 64, 256, 20)])
def test_log_prob_at_workload_shapes(gpu, orc, L, C, B, n_check):
    """The learned workloads' shapes (L = 32, 32 channels, batches of 4096; L =
    64, 64 channels, 256 chains), the whole batch on the GPU, the oracle on a
    sample of it that includes equilibrium Ising configurations."""
    say(f"log_prob workload L={L} C={C} B={B}")
    th = bf16_params(C, 7 * L, scale=1.0)
    x = mixed_configs(B, L, 500 + L, orc, n_ising=n_check // 2)
    idx = np.concatenate([np.arange(n_check // 2),
                          np.random.default_rng(L).choice(np.arange(n_check // 2, B),
                                                          n_check - n_check // 2, replace=False)])
    check_log_prob(gpu, L, C, B, th, x, idx)


def serial_terms(B, L, C):
    rows = B * L * L
    nchunks = (rows + 63) // 64
    nblk = min(256, nchunks)
    cpb = (nchunks + nblk - 1) // nblk
    return 64 * cpb + nblk + 25 * C


def grad_bound(G, B, L, C):
    return (2.0 ** -15 + serial_terms(B, L, C) * U_F32) * G


GRAD_SHAPES = [(8, 32, 12), (8, 64, 12), (32, 32, 256), (64, 64, 16)]


@pytest.mark.parametrize("L,C,B", GRAD_SHAPES)
def test_gradient_at_given_activations_elementwise(gpu, L, C, B):
    """Every gradient element of the backward pass at seeded activations and
    logits against the double backward pass (signal unrounded); (32, 32, 256)
    is a training batch of the L = 32 workload."""
    import torch

    say(f"gradient at given activations L={L} C={C} B={B}")
    th = bf16_params(C, 5 + L, scale=1.0)
    x = mixed_configs(B, L, 60 + L)
    rng = np.random.default_rng(70 + L)
    acts = [ref.bf16(np.maximum(rng.normal(0.1, 1.0, (B, L, L, C)), 0.0)) for _ in range(5)]
    z = rng.normal(0, 2.0, (B, L, L)).astype(np.float32).astype(np.float64)
    net = gpu.ARNet(L, C, B)
    net.set_params(th.astype(np.float32))
    d_acts = torch.as_tensor(np.stack(acts).astype(np.float32)).to(torch.bfloat16).cuda().contiguous()
    loss, g = net.gradient_at(spins_t(x), d_acts, torch.as_tensor(z.astype(np.float32)).cuda())
    nll, want = ref.backward_from(x, z, acts, th, C)
    S = serial_terms(B, L, C)
    assert abs(float(loss.item()) - nll) <= (S + 520) * U_F32 * abs(nll), (float(loss.item()), nll)
    got = g.cpu().numpy().astype(np.float64)
    bound = grad_bound(ref.grad_abs_from(x, z, acts, th, C), B, L, C)
    err = np.abs(got - want)
    ratio = err / np.maximum(bound, 1e-300)
    worst = int(np.argmax(ratio))
    say(f"  max |dg|/bound {ratio[worst]:.3g} (element {worst})")
    assert np.all(err <= bound), (worst, got[worst], want[worst], bound[worst])
    net.close()


@pytest.mark.parametrize("L,C,B", GRAD_SHAPES)
def test_gradient_end_to_end(gpu, L, C, B):
    """Forward and backward on the GPU against the double oracle of the
    network with bf16-stored activations (see the module docstring)."""
    say(f"gradient end to end L={L} C={C} B={B}")
    th = bf16_params(C, 5 + L, scale=1.0)
    x = mixed_configs(B, L, 60 + L)
    net = gpu.ARNet(L, C, B)
    net.set_params(th.astype(np.float32))
    loss, g = net.gradient(spins_t(x))
    nll, want = ref.nll_and_grad(x, th, C, emulate_bf16=True)
    assert abs(float(loss.item()) - nll) <= 1e-4 * abs(nll), (float(loss.item()), nll)
    got = g.cpu().numpy().astype(np.float64)
    G = ref.grad_abs(x, th, C)
    err = np.abs(got - want)
    within = err <= grad_bound(G, B, L, C)
    worst = float(np.max(err / np.maximum(G, 1e-300)))
    say(f"  {within.mean():.5f} of elements within the tight bound; max |dg|/G^abs {worst:.3g}")
    assert within.mean() >= 0.99
    assert np.all(err <= 2.0 ** -5 * G)
    net.close()


def test_gradients_and_training_are_reproducible(gpu):
    """Fixed-order sums: the same gradient twice, and two networks trained
    from the same start on the same batches end bit-identical."""
    import torch

    L, C, B = 16, 32, 64
    th = ref.init_params(C, 3, scale=0.7).astype(np.float32)
    data = spins_t(mixed_configs(4 * B, L, 9))
    nets = [gpu.ARNet(L, C, B) for _ in range(2)]
    for n in nets:
        n.set_params(th)
    _, g1 = nets[0].gradient(data[:B].contiguous())
    _, g2 = nets[0].gradient(data[:B].contiguous())
    assert torch.equal(g1, g2)
    losses = [[], []]
    for k, n in enumerate(nets):
        for s in range(12):
            xb = data[(s % 4) * B:(s % 4 + 1) * B].contiguous()
            losses[k].append(float(n.train_step(xb, 2e-3).item()))
    assert losses[0] == losses[1]
    assert torch.equal(nets[0].params(), nets[1].params())
    for n in nets:
        n.close()


@pytest.mark.parametrize("C,L,B", [(32, 8, 37), (64, 6, 37), (32, 16, 37), (32, 32, 4096),
                                   (64, 64, 256), (32, 2, 5), (32, 3, 7)])
def test_sampler_matches_evaluator_and_uniforms(gpu, C, L, B):
    """The sampler's log q~ equals the evaluator's bit for bit on the drawn
    configurations; each drawn spin is +1 exactly when its domain-3 uniform
    is below the conditional of the oracle's bf16-storage forward pass (sites
    whose uniform lies within SAMPLE_MARGIN of it are not judged: a float32
    forward pass rounds a few activations to the other neighbouring bf16
    value, which moves conditionals downstream of them by up to ~1e-3);
    rounds and streams select other draws."""
    say(f"sampler C={C} L={L} B={B}")
    th = bf16_params(C, 40 + L, scale=1.5)
    net = gpu.ARNet(L, C, B)
    net.set_params(th.astype(np.float32))
    seed, sb, rnd = 11, 5, 3
    x, lq = net.sample(B, seed=seed, stream_base=sb, round=rnd)
    lq2 = net.log_prob(x)
    assert np.array_equal(lq.cpu().numpy(), lq2.cpu().numpy())
    xs = x.cpu().numpy()
    assert set(np.unique(xs)) <= {-1, 1}
    n_judge = min(B, 8)
    xj = xs[:n_judge].astype(np.float64)
    z, _ = ref.forward(xj, th, C, emulate_bf16=True)
    Pq = ref.quantised_p(z)
    judged = wrong = 0
    for c in range(n_judge):
        u = ref.sample_uniforms(seed, sb + c, rnd, L * L).reshape(L, L)
        clear = np.abs(u - Pq[c]) > SAMPLE_MARGIN
        want = np.where(u < Pq[c], 1, -1)
        judged += int(clear.sum())
        wrong += int((xs[c][clear] != want[clear]).sum())
    say(f"  {judged} of {n_judge * L * L} draws judged, {wrong} differ")
    assert wrong == 0 and judged >= 0.95 * n_judge * L * L
    x_same, _ = net.sample(B, seed=seed, stream_base=sb, round=rnd)
    x_other, _ = net.sample(B, seed=seed, stream_base=sb, round=rnd + 1)
    assert np.array_equal(x_same.cpu().numpy(), xs)
    if L >= 4:
        assert not np.array_equal(x_other.cpu().numpy(), xs)
    net.close()


@pytest.mark.parametrize("C,L,B", [(32, 2, 5), (32, 3, 7), (64, 6, 37), (32, 8, 37),
                                   (64, 16, 40), (32, 16, 100), (32, 32, 4096), (64, 64, 64)])
def test_on_chip_evaluator_equals_layer_kernels(gpu, C, L, B):
    """log q~ and the logits of the on-chip evaluator (one workgroup per
    configuration, activations in LDS) equal those of the one-launch-per-layer
    path bit for bit, partial last tiles (L*L not a multiple of 16) included;
    at L = 64, C = 64 the activations do not fit and both modes take the layer
    kernels."""
    say(f"evaluators C={C} L={L} B={B}")
    th = bf16_params(C, 60 + L, scale=1.0)
    x = spins_t(mixed_configs(B, L, 900 + L))
    net = gpu.ARNet(L, C, B)
    net.set_params(th.astype(np.float32))
    q_auto, z_auto = net.log_prob(x, logits=True)
    q_only = net.log_prob(x)
    net.set_eval_mode("layers")
    q_lay, z_lay = net.log_prob(x, logits=True)
    net.set_eval_mode("auto")
    q_auto2 = net.log_prob(x)
    a, b = q_auto.cpu().numpy(), q_lay.cpu().numpy()
    assert not np.any(np.isnan(a)) and np.mean(np.isfinite(a)) > 0.5
    assert np.array_equal(a, b), np.flatnonzero(a != b)[:5]
    assert np.array_equal(z_auto.cpu().numpy(), z_lay.cpu().numpy())
    assert np.array_equal(q_only.cpu().numpy(), a) and np.array_equal(q_auto2.cpu().numpy(), a)
    net.close()


def test_eval_mode_rejects_unknown_values(gpu):
    lib = gpu._lib.load()
    net = gpu.ARNet(4, 32, 1)
    assert lib.ising_arnet_set_eval_mode(net._h, 2) != 0
    assert lib.ising_arnet_set_eval_mode(net._h, -1) != 0
    assert lib.ising_arnet_set_eval_mode(net._h, 1) == 0
    net.close()


def test_sampler_rejects_lattices_beyond_its_lds(gpu):
    import torch

    net = gpu.ARNet(130, 32, 1)
    with pytest.raises(Exception):
        net.sample(1, seed=1)
    torch.cuda.synchronize()
    net.close()


def test_sampling_frequencies_match_q(gpu):
    C, L, n = 32, 2, 1 << 16
    th = bf16_params(C, 77, scale=2.0)
    net = gpu.ARNet(L, C, n)
    net.set_params(th.astype(np.float32))
    x, lq = net.sample(n, seed=3)
    xs = x.cpu().numpy().reshape(n, -1)
    codes = ((xs > 0) * (1 << np.arange(L * L))).sum(axis=1)
    states = exact.all_states(L).astype(np.float64)
    q = np.exp(ref.log_q_exact(states, th, C, emulate_bf16=False))
    assert abs(q.sum() - 1) < 1e-9
    counts = np.bincount(codes, minlength=16)
    sd = np.sqrt(n * q * (1 - q))
    assert np.all(np.abs(counts - n * q) <= 5 * sd + 2), (counts, n * q)
    net.close()


def test_mh_decisions_match_oracle(gpu, orc):
    """Independence MH on 4096 chains: every decision equals the oracle's
    float32 rule with the oracle's domain-2 uniforms (chains whose uniform
    lies within 4 ulps of exp(log A) may go either way and are counted), and
    accepted chains take the proposal's spins, log q~ and bond sum."""
    import torch

    n, L = 4096, 8
    rng = np.random.default_rng(21)
    for rnd in (1, 2, 7):
        state = rand_spins(n, L, 100 + rnd, 0.6)
        prop = rand_spins(n, L, 200 + rnd, 0.4)
        bond = np.array([orc.observables(s)[0] for s in state], dtype=np.int64)
        bond_p = np.array([orc.observables(s)[0] for s in prop], dtype=np.int64)
        lq = rng.uniform(-60, -40, n).astype(np.float32)
        lqp = rng.uniform(-60, -40, n).astype(np.float32)
        betaJ = np.full(n, 0.44, dtype=np.float32)
        d_state, d_prop = spins_t(state), spins_t(prop)
        d_lq = torch.as_tensor(lq).cuda()
        d_bond = torch.as_tensor(bond).cuda()
        acc = gpu.mh_independence(d_state, d_lq, d_bond, d_prop, torch.as_tensor(lqp).cuda(),
                                  torch.as_tensor(bond_p).cuda(), torch.as_tensor(betaJ).cuda(),
                                  seed=9, stream_base=0, round=rnd)
        got = acc.cpu().numpy().astype(bool)
        want, amb = ref.mh_decisions(bond, bond_p, lq, lqp, betaJ, seed=9, stream_base=0, rnd=rnd)
        say(f"  round {rnd}: acceptance {got.mean():.3f}, {int(amb.sum())} ambiguous")
        assert amb.sum() <= 3
        assert np.array_equal(got[~amb], want[~amb])
        exp_state = np.where(got[:, None, None], prop, state)
        assert np.array_equal(d_state.cpu().numpy(), exp_state)
        assert np.array_equal(d_lq.cpu().numpy(), np.where(got, lqp, lq))
        assert np.array_equal(d_bond.cpu().numpy(), np.where(got, bond_p, bond))


def test_adam_matches_oracle(gpu):
    """Four Adam steps with given gradients against the double-precision
    update with the same (float32) constants; float32 rounds each of about ten
    operations per step, so the parameters agree within
    steps * (2^-23 |theta| + 2^-20 lr)."""
    import torch

    C, L = 32, 8
    P = ref.num_params(C)
    rng = np.random.default_rng(31)
    th = rng.normal(0, 0.3, P)
    net = gpu.ARNet(L, C, 1)
    net.set_params(th.astype(np.float32))
    th_ref = th.astype(np.float32).astype(np.float64)
    m = np.zeros(P)
    v = np.zeros(P)
    lr = 1e-2
    for k in range(1, 5):
        g = (rng.normal(size=P) * 10.0 ** rng.uniform(-4, 0, P)).astype(np.float32)
        net.adam(torch.as_tensor(g).cuda(), lr)
        th_ref, m, v = ref.adam_step(th_ref, g.astype(np.float64), m, v, k, lr,
                                     beta1=float(np.float32(0.9)), beta2=float(np.float32(0.999)),
                                     eps=float(np.float32(1e-8)))
        got = net.params().cpu().numpy().astype(np.float64)
        tol = k * (2.0 ** -23 * np.abs(th_ref) + 2.0 ** -20 * lr)
        assert np.all(np.abs(got - th_ref) <= tol), (k, np.max(np.abs(got - th_ref) / tol))
    net.close()


@pytest.mark.parametrize("L,B", [(4, 50), (6, 33), (32, 4096), (64, 256)])
def test_spins_observables_match_oracle(gpu, orc, L, B):
    x = mixed_configs(B, L, 40 + L)
    bond, mag = gpu.spins_observables(spins_t(x), L)
    want = np.array([orc.observables(s) for s in x], dtype=np.int64)
    assert np.array_equal(bond.cpu().numpy(), want[:, 0])
    assert np.array_equal(mag.cpu().numpy(), want[:, 1])


@pytest.mark.parametrize("L,P,B", [(6, 40, 300), (32, 1000, 256), (64, 100, 64)])
def test_minibatch_matches_oracle(gpu, L, P, B):
    """Training minibatches (pool member, flip and translation from Philox
    domain 5) bit for bit against the oracle's draw."""
    pool = mixed_configs(P, L, 80 + L)
    d_pool = spins_t(pool)
    for rnd in (0, 1, 12345678901):
        got = gpu.spins_minibatch(d_pool, B, seed=77, stream_base=9, round=rnd).cpu().numpy()
        assert np.array_equal(got, ref.augmented_minibatch(pool, B, 77, 9, rnd)), rnd


def test_independence_chain_exact_on_4x4(gpu):
    """Learned-proposal Metropolis-Hastings keeps the Boltzmann distribution:
    chains started from exact 4x4 Boltzmann samples stay there (random-weight
    q, pure global moves); averages within 3 standard errors of enumeration."""
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
        assert abs(per_chain.mean() - target) < 3 * se, (per_chain.mean(), target, se)
    net.close()


def test_training_lowers_the_loss(gpu, orc):
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
