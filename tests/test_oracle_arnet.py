"""Pins of the autoregressive-proposal oracle: hand-written gradient against
double-precision finite differences and against PyTorch autograd (also of the
bf16-rounded network, straight-through), the autoregressive property,
normalisation by enumeration, exactness of the independence
Metropolis-Hastings chain on 4x4 against enumeration, the absolute-value
scales used by the GPU tolerances, Adam's closed forms, and the addressing
and frequencies of the sampling and acceptance uniforms."""
import numpy as np
import pytest

from oracle import arnet, exact, stats


def rand_spins(B, L, seed):
    return np.where(np.random.default_rng(seed).random((B, L, L)) < 0.5, 1.0, -1.0)


def test_param_count_and_roundtrip():
    for C in (1, 3, 32, 64):
        th = arnet.init_params(C, 1)
        assert th.size == arnet.num_params(C)
        assert np.array_equal(arnet.flatten(arnet.unflatten(th, C), C), th)


def test_gradient_matches_finite_differences():
    C, L = 3, 5
    th = arnet.init_params(C, 7, scale=1.3) + np.random.default_rng(8).normal(0, 0.2, arnet.num_params(C))
    x = rand_spins(4, L, 9)
    _, g = arnet.nll_and_grad(x, th, C)
    rng = np.random.default_rng(10)
    idx = rng.choice(th.size, 60, replace=False)
    h = 1e-6
    for k in idx:
        e = np.zeros_like(th)
        e[k] = h
        num = (arnet.nll_and_grad(x, th + e, C)[0] - arnet.nll_and_grad(x, th - e, C)[0]) / (2 * h)
        assert abs(num - g[k]) <= 1e-6 + 1e-5 * abs(num), (k, num, g[k])


def _torch_bf16(t):
    """Straight-through bfloat16 rounding: the forward value is rounded (the
    oracle's own bf16() of the detached tensor), the derivative is 1."""
    import torch

    r = torch.tensor(arnet.bf16(t.detach().numpy()))
    return t + (r - t).detach()


@pytest.mark.parametrize("emulate", [False, True])
def test_gradient_matches_torch_autograd(emulate):
    """The hand-written backward against PyTorch CPU autograd: of the plain
    network, and (emulate) of the network with weights and stored activations
    rounded to bfloat16, the rounding taken as the identity in the backward
    pass, the backward signal unrounded."""
    torch = pytest.importorskip("torch")
    C, L = 4, 6
    th = arnet.init_params(C, 3) + np.random.default_rng(4).normal(0, 0.1, arnet.num_params(C))
    x = rand_spins(5, L, 5)
    nll, g = arnet.nll_and_grad(x, th, C, emulate_bf16=emulate)
    p = {k: torch.tensor(np.asarray(v, dtype=np.float64), requires_grad=True) for k, v in arnet.unflatten(th, C).items()}
    rw = _torch_bf16 if emulate else (lambda t: t)
    xt = torch.tensor(x)[:, None]  # (B, 1, L, L)

    def masked_conv(h, taps_w, bias):
        # taps_w: list of (dy, dx, [cin, cout]) ; out[b, co, i, j] = sum h[b, ci, i+dy, j+dx] w[ci, co]
        out = 0
        for (dy, dx), w in taps_w:
            hp = torch.nn.functional.pad(h, (1, 1, 1, 1))
            hs = hp[:, :, 1 + dy:1 + dy + L, 1 + dx:1 + dx + L]
            out = out + torch.einsum("bcij,cd->bdij", hs, w)
        return out + bias.reshape(1, -1, 1, 1)

    h = rw(torch.relu(masked_conv(xt, [(arnet.TAPS[t], rw(p["W1"][t])[None, :]) for t in range(4)], p["b1"])))
    for l in range(2, 6):
        h = rw(torch.relu(masked_conv(h, [(arnet.TAPS[t], rw(p[f"W{l}"][t])) for t in range(5)], p[f"b{l}"])))
    logit = masked_conv(h, [(arnet.TAPS[t], rw(p["W6"][t])[:, None]) for t in range(5)], p["b6"].reshape(1))[:, 0]
    loss = -torch.nn.functional.logsigmoid(torch.tensor(x) * logit).sum() / x.shape[0]
    loss.backward()
    gt = arnet.flatten({k: v.grad.numpy() for k, v in p.items()}, C)
    assert abs(float(loss.detach()) - nll) < 1e-10
    assert np.allclose(gt, g, rtol=1e-9, atol=1e-12)


def test_autoregressive_property():
    """logit_p depends only on sites strictly before p in raster order."""
    C, L = 4, 6
    th = arnet.init_params(C, 11, scale=1.5)
    x = rand_spins(1, L, 12)
    base, _ = arnet.forward(x, th, C)
    for site in range(L * L):
        y = x.copy()
        y[0, site // L, site % L] *= -1
        logit, _ = arnet.forward(y, th, C)
        diff = (logit != base).reshape(-1)
        assert not diff[: site + 1].any(), site  # sites <= the flipped one unchanged


@pytest.mark.parametrize("emulate", [False, True])
def test_normalisation_by_enumeration(emulate):
    C, L = 3, 4
    th = arnet.init_params(C, 21, scale=2.0)
    states = exact.all_states(L).astype(np.float64)
    lq = arnet.log_q(states, th, C, emulate)
    assert abs(np.exp(lq).sum() - 1.0) < 1e-12
    lqe = arnet.log_q_exact(states, th, C, emulate)
    assert abs(np.exp(lqe).sum() - 1.0) < 1e-9


def test_sampler_frequencies_match_q():
    C, L = 2, 2  # 16 states: compare empirical frequencies with q_exact
    th = arnet.init_params(C, 5, scale=2.0)
    rng = np.random.default_rng(6)
    x, lq = arnet.sample(th, C, L, 40000, rng)
    assert np.allclose(lq, arnet.log_q_exact(x, th, C), atol=1e-9)
    codes = ((x.reshape(len(x), -1) > 0) * (1 << np.arange(L * L))).sum(axis=1)
    states = exact.all_states(L).astype(np.float64)
    q = np.exp(arnet.log_q_exact(states, th, C))
    counts = np.bincount(codes, minlength=16)
    sd = np.sqrt(len(x) * q * (1 - q))
    assert np.all(np.abs(counts - len(x) * q) <= 5 * sd + 1)


def test_independence_chain_is_exact_on_4x4():
    """A chain of pure learned proposals with a random-weight q reproduces the
    Boltzmann averages (q has full support; MH corrects for it).  A random q is
    nearly uniform over the 65536 states, so the temperature is chosen where
    30000 proposals mix (at beta_c the few ordered states that carry most of
    the weight are hardly ever proposed)."""
    C, L, beta = 2, 4, 0.25
    th = arnet.init_params(C, 33, scale=0.6)
    rng = np.random.default_rng(34)
    nprop = 30000
    xs, lqs = arnet.sample(th, C, L, nprop, rng)
    bonds = exact.bond_sum_many(xs.astype(np.int8)).astype(np.float64)
    cur = 0
    E, M2 = np.empty(nprop), np.empty(nprop)
    acc = 0
    u = rng.random(nprop)
    for k in range(1, nprop):
        a = arnet.mh_accept_prob(beta, 1.0, bonds[cur], bonds[k], lqs[cur], lqs[k])
        if u[k] < a:
            cur = k
            acc += 1
        E[k] = -bonds[cur] / 16
        M2[k] = (xs[cur].sum() / 16) ** 2
    E, M2 = E[100:], M2[100:]
    ex = exact.enumerate_lattice(L, beta)
    assert acc > 1000
    for s, target in ((E, ex["E_per_site"]), (M2, ex["m2"])):
        se = stats.blocking_se(s)
        assert abs(s.mean() - target) < 4.5 * se, (s.mean(), target, se)


def test_abs_scales_bound_and_are_attained():
    """forward_abs bounds |logit| and grad_abs bounds |gradient| element by
    element; with non-negative weights and biases, all spins +1, every product
    has one sign and both are attained exactly."""
    C, L = 3, 5
    th = arnet.init_params(C, 13, scale=1.4) + np.random.default_rng(14).normal(0, 0.1, arnet.num_params(C))
    x = rand_spins(3, L, 15)
    z, _ = arnet.forward(x, th, C, emulate_bf16=True)
    assert np.all(np.abs(z) <= arnet.forward_abs(x, arnet.bf16(th), C) * (1 + 1e-12))
    _, g = arnet.nll_and_grad(x, th, C, emulate_bf16=True)
    assert np.all(np.abs(g) <= arnet.grad_abs(x, th, C) * (1 + 1e-12) + 1e-300)
    pos = np.abs(th)
    ones = np.ones((2, L, L))
    z, _ = arnet.forward(ones, pos, C)
    assert np.allclose(arnet.forward_abs(ones, pos, C), np.abs(z), rtol=1e-13)
    _, g = arnet.nll_and_grad(ones, pos, C)
    assert np.allclose(arnet.grad_abs(ones, pos, C, emulate_bf16=False), np.abs(g), rtol=1e-12,
                       atol=1e-300)


def test_adam_closed_forms():
    """First step: m^ = g, v^ = g^2, so theta moves by lr g / (|g| + eps); a
    constant gradient keeps m^ = g and v^ = g^2 at every step (the bias
    corrections undo the zero start)."""
    rng = np.random.default_rng(16)
    th0 = rng.normal(size=50)
    g = rng.normal(size=50) * 10.0 ** rng.uniform(-3, 1, 50)
    lr, eps = 1e-3, 1e-8
    th, m, v = arnet.adam_step(th0, g, np.zeros(50), np.zeros(50), 1, lr, eps=eps)
    step = lr * g / (np.abs(g) + eps)
    assert np.allclose(th0 - th, step, rtol=1e-12, atol=0)
    for k in range(2, 12):
        prev = th
        th, m, v = arnet.adam_step(th, g, m, v, k, lr, eps=eps)
        assert np.allclose(prev - th, step, rtol=1e-9, atol=0)
    # a zero gradient never moves a parameter
    th2, _, _ = arnet.adam_step(th0, np.zeros(50), np.zeros(50), np.zeros(50), 1, lr)
    assert np.array_equal(th2, th0)


def test_sampling_uniforms_address_the_generator():
    """u_p of site p is word p & 3 of the block at counter word 3 = p >> 2,
    scaled 24 bits; distinct streams and rounds give distinct draws."""
    import oracle

    seed, stream, rnd, N = 0x123456789, 77, (5 << 32) | 9, 10
    u = arnet.sample_uniforms(seed, stream, rnd, N)
    for p in range(N):
        blk = oracle.philox4x32_10(((stream << 8) | (3 << 4), 9, 5, p >> 2),
                                   (seed & 0xFFFFFFFF, seed >> 32))
        assert u[p] == (blk[p & 3] >> 8) / 2.0 ** 24
    assert not np.array_equal(u, arnet.sample_uniforms(seed, stream + 1, rnd, N))
    assert not np.array_equal(u, arnet.sample_uniforms(seed, stream, rnd + 1, N))
    big = arnet.sample_uniforms(3, 0, 0, 40000)
    assert np.all((big >= 0) & (big < 1))
    assert abs(big.mean() - 0.5) < 4 * np.sqrt(1 / 12 / big.size)


def test_mh_decisions_rule_and_frequency():
    """log A >= 0 always accepts; at a fixed log A = ln a the accepted fraction
    over independent streams is a (binomial error); the float32 ratio is
    ((beta J dB) + log q) - log q'."""
    n = 20000
    a = 0.3
    la = np.float32(np.log(a))
    acc, amb = arnet.mh_decisions(np.zeros(n), np.zeros(n), np.full(n, la), np.zeros(n),
                                  np.zeros(n), seed=5, stream_base=0, rnd=3)
    assert abs(acc.mean() - a) < 4 * np.sqrt(a * (1 - a) / n)
    assert amb.sum() <= 4
    acc, amb = arnet.mh_decisions(np.zeros(8), np.full(8, 4), np.full(8, -10.0), np.full(8, -9.0),
                                  np.full(8, 0.25), seed=5, stream_base=0, rnd=3)
    assert acc.all() and not amb.any()  # 0.25 * 4 - 10 + 9 = 0 >= 0
    acc, _ = arnet.mh_decisions(np.zeros(8), np.full(8, -400), np.zeros(8), np.zeros(8),
                                np.full(8, 0.25), seed=5, stream_base=0, rnd=3)
    assert not acc.any()  # A = e^-100



def test_backward_from_given_activations_is_the_backward_pass():
    """backward_from on the forward pass's own logits and activations is
    nll_and_grad; on other activations its W6 and b6 parts are the plain
    contractions of the definition (spot-checked by brute force)."""
    C, L, B = 3, 5, 4
    th = arnet.init_params(C, 41, scale=1.1) + np.random.default_rng(42).normal(0, 0.1, arnet.num_params(C))
    x = rand_spins(B, L, 43)
    z, acts = arnet.forward(x, th, C, emulate_bf16=True)
    assert np.array_equal(arnet.backward_from(x, z, acts, th, C)[1],
                          arnet.nll_and_grad(x, th, C, emulate_bf16=True)[1])
    rng = np.random.default_rng(44)
    acts2 = [np.maximum(rng.normal(size=a.shape), 0) for a in acts]
    z2 = rng.normal(size=z.shape)
    nll, g = arnet.backward_from(x, z2, acts2, th, C)
    dl = -x / (1 + np.exp(x * z2)) / B
    gW6 = arnet.unflatten(g, C)["W6"]
    for t, (dy, dx) in enumerate(arnet.TAPS):
        want = np.zeros(C)
        for b in range(B):
            for i in range(L):
                for j in range(L):
                    if 0 <= i + dy < L and 0 <= j + dx < L:
                        want += acts2[4][b, i + dy, j + dx] * dl[b, i, j]
        assert np.allclose(gW6[t], want, rtol=1e-12, atol=1e-15)
    assert abs(float(arnet.unflatten(g, C)["b6"]) - dl.sum()) < 1e-14
    assert abs(nll - np.logaddexp(0, -x * z2).sum() / B) < 1e-12
    G = arnet.grad_abs_from(x, z2, acts2, th, C)
    assert np.all(np.abs(g) <= G * (1 + 1e-12) + 1e-300)


def test_augmented_minibatch_draws_symmetry_images():
    """Every drawn configuration is a flip and translation of a pool member,
    keeps that member's bond sum (the Boltzmann weight), and over many draws
    members, flips and shifts are uniform (chi-squared)."""
    from oracle import exact

    rng = np.random.default_rng(50)
    P, L, B = 8, 6, 4000
    pool = np.where(rng.random((P, L, L)) < 0.5, 1, -1).astype(np.int8)
    pool[0] = 1  # an all-up member: its images are all-up or all-down
    out = arnet.augmented_minibatch(pool, B, seed=0x1234567890, stream_base=3, rnd=7)
    bond = exact.bond_sum_many(pool)
    images = {}
    for k in range(P):
        for f in (1, -1):
            for di in range(L):
                for dj in range(L):
                    y = f * np.roll(pool[k], shift=(-di, -dj), axis=(0, 1))
                    images.setdefault(y.tobytes(), (k, f, di, dj))
    ks, fs, dis, djs = [], [], [], []
    for b in range(B):
        k, f, di, dj = images[out[b].tobytes()]
        assert exact.bond_sum_many(out[b:b + 1])[0] == bond[k]
        ks.append(k)
        fs.append(f)
        if k != 0:
            dis.append(di)
            djs.append(dj)
    for vals, m in ((ks, P), (dis, L), (djs, L)):
        c = np.bincount(vals, minlength=m)
        e = len(vals) / m
        assert ((c - e) ** 2 / e).sum() < 3 * m  # loose chi-squared bound, m - 1 dof
    assert abs(np.mean(np.array(fs) > 0) - 0.5) < 4 * np.sqrt(0.25 / B)
    again = arnet.augmented_minibatch(pool, 5, seed=0x1234567890, stream_base=3, rnd=7)
    assert np.array_equal(again, out[:5])
    assert not np.array_equal(arnet.augmented_minibatch(pool, 5, 0x1234567890, 3, 8), out[:5])
