"""Oracle of the learned global proposal: a masked-convolution autoregressive
network over Ising configurations and the independence Metropolis-Hastings
step that uses it.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper motivates global moves by critical slowing down of local Metropolis
updates and by the Wolff cluster algorithm (Sec. 2); it does not specify a
learned proposal.  The network here is the standard PixelCNN construction
(van den Oord et al., "Pixel Recurrent Neural Networks", ICML 2016), with the
readings fixed for this project:

  * sites in raster order p = i*L + j; the model is
        q(x) = prod_p  q(x_p | x_<p),   q(x_p = +1 | x_<p) = sigmoid(logit_p);
  * layer 1: 3x3 convolution with mask "A" (only strictly earlier sites:
    offsets (-1,-1), (-1,0), (-1,+1), (0,-1)), 1 -> C channels, ReLU;
  * layers 2..5: 3x3 mask "B" (those four offsets and the centre), C -> C, ReLU;
  * layer 6: mask "B", C -> 1, giving the logit of every site;
  * zero padding outside the lattice (no periodic wrap), so the conditionals
    depend only on earlier sites.

Parameters, in this order (the flat vector used everywhere):
    W1[4][C], b1[C], (W_l[5][C][C], b_l[C]) for l = 2..5, W6[5][C], b6.
W_l[t][ci][co] multiplies input channel ci at tap offset t into output co.

Sampling draws x_p = +1 iff u_p < P_p with u_p a 24-bit uniform, so the
realised probability of +1 is P~_p = ceil(P_p * 2^24) / 2^24, and the exact
proposal probability of a configuration is prod_p (P~_p or 1 - P~_p).
``log_q_exact`` computes that; ``log_q`` the smooth model value used by training.
"""
from __future__ import annotations

import numpy as np

TAPS = ((-1, -1), (-1, 0), (-1, 1), (0, -1), (0, 0))  # mask A = first four
N_LAYERS = 6


def num_params(C: int) -> int:
    return 4 * C + C + 4 * (5 * C * C + C) + 5 * C + 1


def unflatten(theta: np.ndarray, C: int) -> dict:
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == num_params(C)
    out, o = {}, 0

    def take(shape):
        nonlocal o
        n = int(np.prod(shape))
        v = theta[o:o + n].reshape(shape)
        o += n
        return v

    out["W1"], out["b1"] = take((4, C)), take((C,))
    for l in range(2, 6):
        out[f"W{l}"], out[f"b{l}"] = take((5, C, C)), take((C,))
    out["W6"], out["b6"] = take((5, C)), take(())
    return out


def flatten(p: dict, C: int) -> np.ndarray:
    parts = [p["W1"], p["b1"]]
    for l in range(2, 6):
        parts += [p[f"W{l}"], p[f"b{l}"]]
    parts += [p["W6"], np.atleast_1d(p["b6"])]
    return np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1) for a in parts])


def init_params(C: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """He-style random parameters (fan-in = taps x input channels)."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.normal(0, scale * np.sqrt(2 / 4), (4, C)), "b1": np.zeros(C)}
    for l in range(2, 6):
        p[f"W{l}"] = rng.normal(0, scale * np.sqrt(2 / (5 * C)), (5, C, C))
        p[f"b{l}"] = np.zeros(C)
    p["W6"] = rng.normal(0, scale * np.sqrt(1 / (5 * C)), (5, C))
    p["b6"] = np.float64(0.0)
    return flatten(p, C)


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) and back, via float32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shift(h: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """out[b, i, j, ...] = h[b, i+dy, j+dx, ...], zero outside the lattice."""
    out = np.zeros_like(h)
    L = h.shape[1]
    i0, i1 = max(0, -dy), min(L, L - dy)
    j0, j1 = max(0, -dx), min(L, L - dx)
    out[:, i0:i1, j0:j1] = h[:, i0 + dy:i1 + dy, j0 + dx:j1 + dx]
    return out


def forward(x: np.ndarray, theta: np.ndarray, C: int, emulate_bf16: bool = False):
    """logits [B, L, L] and the list of activations (post-ReLU) of layers 1..5.

    emulate_bf16: round weights, and activations between layers, to bfloat16
    where the GPU stores them (sums stay in double)."""
    p = unflatten(theta, C)
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    acts = []
    pre = np.zeros(x.shape + (C,))
    for t in range(4):
        pre += shift(x, *TAPS[t])[..., None] * r(p["W1"][t])[None, None, None, :]
    h = r(np.maximum(pre + p["b1"], 0.0))
    acts.append(h)
    for l in range(2, 6):
        W = r(p[f"W{l}"])
        pre = np.zeros_like(h)
        for t in range(5):
            pre += _apply_right(shift(h, *TAPS[t]), W[t])
        h = r(np.maximum(pre + p[f"b{l}"], 0.0))
        acts.append(h)
    W6 = r(p["W6"])
    logit = np.full(x.shape, float(p["b6"]))
    for t in range(5):
        logit += np.einsum("bijc,c->bij", shift(h, *TAPS[t]), W6[t])
    return logit, acts


def log_sigmoid(z):
    return -np.logaddexp(0.0, -z)


def log_q(x, theta, C, emulate_bf16=False) -> np.ndarray:
    """Model log-probability sum_p log sigmoid(x_p * logit_p), per configuration."""
    logit, _ = forward(x, theta, C, emulate_bf16)
    return log_sigmoid(np.asarray(x, np.float64) * logit).sum(axis=(1, 2))


def quantised_p(logit: np.ndarray) -> np.ndarray:
    """P~ = ceil(P * 2^24) / 2^24 with P = sigmoid(logit) in float32."""
    P = (1.0 / (1.0 + np.exp(-np.asarray(logit, dtype=np.float32)))).astype(np.float32)
    return np.ceil(P.astype(np.float64) * 2.0 ** 24) / 2.0 ** 24


def log_q_exact(x, theta, C, emulate_bf16=True) -> np.ndarray:
    """Exact log-probability that the sampler produces x (24-bit uniforms)."""
    logit, _ = forward(x, theta, C, emulate_bf16)
    Pq = quantised_p(logit)
    x = np.asarray(x)
    with np.errstate(divide="ignore"):
        terms = np.where(x > 0, np.log(Pq), np.log1p(-Pq))
    return terms.sum(axis=(1, 2))


def nll_and_grad(x: np.ndarray, theta: np.ndarray, C: int, emulate_bf16: bool = False):
    """Mean negative log-likelihood of a batch and its gradient (hand-written
    backward through the masked convolutions).

    emulate_bf16 selects the forward pass whose gradient is taken (weights and
    stored activations rounded to bfloat16, as ``forward``); the gradient is
    that of the rounded network with the rounding treated as the identity
    (straight-through).  The backward signal itself is never rounded: every
    step of the backward pass is exact in double."""
    logit, acts = forward(x, theta, C, emulate_bf16)
    return backward_from(x, logit, acts, theta, C, emulate_bf16)


def backward_from(x, logit, acts, theta, C: int, bf16_weights: bool = True):
    """The backward pass of the mean NLL from given logits [B, L, L] and
    post-ReLU activations of layers 1..5 ([B, L, L, C] each): ReLU masks are
    acts > 0, weight gradients contract the given activations.  Returns
    (nll, gradient); with bf16_weights the weights are taken rounded."""
    p = unflatten(theta, C)
    r = bf16 if bf16_weights else (lambda a: np.asarray(a, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    logit = np.asarray(logit, dtype=np.float64)
    acts = [np.asarray(a, dtype=np.float64) for a in acts]
    B = x.shape[0]
    s = x
    nll = -log_sigmoid(s * logit).sum() / B
    # d(-log sigmoid(s z))/dz = -s * sigmoid(-s z)
    with np.errstate(over="ignore"):
        dlogit = -s / (1.0 + np.exp(s * logit)) / B
    g = {k: np.zeros_like(np.asarray(v, dtype=np.float64)) for k, v in p.items()}
    g["b6"] = np.float64(dlogit.sum())
    W6 = r(p["W6"])
    h5 = acts[4]
    dh = np.zeros_like(h5)
    for t in range(5):
        dy, dx = TAPS[t]
        g["W6"][t] = np.einsum("bijc,bij->c", shift(h5, dy, dx), dlogit)
        dh += shift(dlogit[..., None] * W6[t][None, None, None, :], -dy, -dx)
    for l in range(5, 1, -1):
        dpre = dh * (acts[l - 1] > 0)
        g[f"b{l}"] = dpre.sum(axis=(0, 1, 2))
        hin = acts[l - 2]
        W = r(p[f"W{l}"])
        dh = np.zeros_like(hin)
        for t in range(5):
            dy, dx = TAPS[t]
            g[f"W{l}"][t] = _contract_rows(shift(hin, dy, dx), dpre)
            dh += shift(_apply_right(dpre, W[t].T), -dy, -dx)
    dpre = dh * (acts[0] > 0)
    g["b1"] = dpre.sum(axis=(0, 1, 2))
    for t in range(4):
        g["W1"][t] = np.einsum("bij,bijc->c", shift(x, *TAPS[t]), dpre)
    return nll, flatten(g, C)


def _apply_right(h: np.ndarray, W: np.ndarray) -> np.ndarray:
    """h[..., c] @ W[c, d] over the trailing axis (one BLAS product)."""
    return (h.reshape(-1, h.shape[-1]) @ W).reshape(h.shape[:-1] + (W.shape[1],))


def _contract_rows(a: np.ndarray, d: np.ndarray) -> np.ndarray:
    """sum over every leading axis of a[..., c] * d[..., e] -> [c, e]."""
    return a.reshape(-1, a.shape[-1]).T @ d.reshape(-1, d.shape[-1])


def forward_abs(x: np.ndarray, theta: np.ndarray, C: int) -> np.ndarray:
    """Scale of every logit for rounding-error bounds: the forward pass with
    every weight, bias and input replaced by its absolute value and no ReLU,
    A_l = |b_l| + sum_t |W_l[t]|^T A_{l-1}(shifted), A_0 = |x|.  A_l bounds
    |h_l| of the exact network and every sum of absolute products formed on
    the way to the logit."""
    p = unflatten(theta, C)
    a = np.abs(np.asarray(x, dtype=np.float64))
    h = np.zeros(a.shape + (C,))
    for t in range(4):
        h += shift(a, *TAPS[t])[..., None] * np.abs(p["W1"][t])[None, None, None, :]
    h += np.abs(p["b1"])
    for l in range(2, 6):
        W = np.abs(p[f"W{l}"])
        nxt = np.zeros_like(h)
        for t in range(5):
            nxt += _apply_right(shift(h, *TAPS[t]), W[t])
        h = nxt + np.abs(p[f"b{l}"])
    out = np.full(a.shape, abs(float(p["b6"])))
    for t in range(5):
        out += _apply_right(shift(h, *TAPS[t]), np.abs(p["W6"][t])[:, None])[..., 0]
    return out


def grad_abs(x: np.ndarray, theta: np.ndarray, C: int, emulate_bf16: bool = True) -> np.ndarray:
    """Scale of every gradient element for rounding-error bounds: the backward
    pass of ``nll_and_grad`` with every weight, activation and backward signal
    replaced by its absolute value (the same ReLU masks), i.e. the sum of the
    absolute values of the products that make up each gradient element."""
    logit, acts = forward(x, theta, C, emulate_bf16)
    return grad_abs_from(x, logit, acts, theta, C, emulate_bf16)


def grad_abs_from(x, logit, acts, theta, C: int, bf16_weights: bool = True) -> np.ndarray:
    """``grad_abs`` of ``backward_from``: from given logits and activations."""
    p = unflatten(theta, C)
    r = bf16 if bf16_weights else (lambda a: np.asarray(a, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    logit = np.asarray(logit, dtype=np.float64)
    acts = [np.asarray(a, dtype=np.float64) for a in acts]
    B = x.shape[0]
    with np.errstate(over="ignore"):
        dlogit = np.abs(1.0 / (1.0 + np.exp(x * logit)) / B)
    g = {k: np.zeros_like(np.asarray(v, dtype=np.float64)) for k, v in p.items()}
    g["b6"] = np.float64(dlogit.sum())
    W6 = np.abs(r(p["W6"]))
    h5 = acts[4]
    dh = np.zeros_like(h5)
    for t in range(5):
        dy, dx = TAPS[t]
        g["W6"][t] = np.einsum("bijc,bij->c", shift(h5, dy, dx), dlogit)
        dh += shift(dlogit[..., None] * W6[t][None, None, None, :], -dy, -dx)
    for l in range(5, 1, -1):
        dpre = dh * (acts[l - 1] > 0)
        g[f"b{l}"] = dpre.sum(axis=(0, 1, 2))
        hin = acts[l - 2]
        W = np.abs(r(p[f"W{l}"]))
        dh = np.zeros_like(hin)
        for t in range(5):
            dy, dx = TAPS[t]
            g[f"W{l}"][t] = _contract_rows(shift(hin, dy, dx), dpre)
            dh += shift(_apply_right(dpre, W[t].T), -dy, -dx)
    dpre = dh * (acts[0] > 0)
    g["b1"] = dpre.sum(axis=(0, 1, 2))
    for t in range(4):
        g["W1"][t] = np.einsum("bij,bijc->c", np.abs(shift(x, *TAPS[t])), dpre)
    return flatten(g, C)


def adam_step(theta, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (Kingma and Ba, ICLR 2015, Algorithm 1) in double:
    m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2, bias corrections
    1 - b1^step and 1 - b2^step, theta <- theta - lr m^ / (sqrt(v^) + eps).
    Returns the new (theta, m, v)."""
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    theta = np.asarray(theta, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return theta, m, v


def mh_accept_prob(beta, J, bond_cur, bond_prop, logq_cur, logq_prop):
    """Independence Metropolis-Hastings acceptance (Metropolis et al. 1953 with
    Hastings' correction): min(1, pi(x') q(x) / (pi(x) q(x'))), pi ~ exp(beta J bond)."""
    log_a = beta * J * (np.asarray(bond_prop) - np.asarray(bond_cur)) + np.asarray(logq_cur) - np.asarray(logq_prop)
    return np.minimum(1.0, np.exp(np.minimum(log_a, 0.0)))


# Counter-based uniforms of the learned part (the same generator as the sweep,
# Philox4x32-10 of SC'11, called through this package's own C copy):
#   domain 2 (Metropolis-Hastings accept): counter (stream<<8 | 2<<4,
#     round mod 2^32, round >> 32, 0), word 0;
#   domain 3 (ancestral sampling, site p): counter (stream<<8 | 3<<4,
#     round mod 2^32, round >> 32, p >> 2), word p & 3;
# each word's top 24 bits give u = k / 2^24.
DOMAIN_MH = 2
DOMAIN_SAMPLE = 3


def _uniform24(seed: int, stream: int, domain: int, rnd: int, c3: int, word: int) -> float:
    from . import philox4x32_10

    ctr = ((stream << 8) | (domain << 4), rnd & 0xFFFFFFFF, (rnd >> 32) & 0xFFFFFFFF, c3)
    out = philox4x32_10(ctr, (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    return (out[word] >> 8) / float(1 << 24)


def sample_uniforms(seed: int, stream: int, rnd: int, N: int) -> np.ndarray:
    """u_p, p = 0..N-1, of one configuration's ancestral draw (domain 3)."""
    from . import philox4x32_10

    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    w0 = (stream << 8) | (DOMAIN_SAMPLE << 4)
    u = np.empty(N)
    for blk in range((N + 3) // 4):
        out = philox4x32_10((w0, rnd & 0xFFFFFFFF, (rnd >> 32) & 0xFFFFFFFF, blk), key)
        for w in range(4):
            if 4 * blk + w < N:
                u[4 * blk + w] = (out[w] >> 8) / float(1 << 24)
    return u


def mh_decisions(bond_cur, bond_prop, logq_cur, logq_prop, betaJ, seed: int, stream_base: int,
                 rnd: int):
    """Independence Metropolis-Hastings decisions (Hastings' ratio for an
    independence proposal, pi ~ exp(beta J bond)) as the reading fixes them:
    in float32, log A = ((betaJ * float(bond' - bond)) + log q(x)) - log q(x'),
    each operation rounded; chain c accepts iff log A >= 0 or u_c < exp(log A),
    u_c the domain-2 uniform of stream stream_base + c.
    Returns (accept, ambiguous): `ambiguous` marks chains whose u_c lies within
    4 float32 ulps of exp(log A), where a faithfully rounded exp may decide
    either way."""
    f32 = np.float32
    dB = (np.asarray(bond_prop, dtype=np.int64) - np.asarray(bond_cur, dtype=np.int64)).astype(f32)
    log_a = ((np.asarray(betaJ, dtype=f32) * dB) + np.asarray(logq_cur, dtype=f32)) \
        - np.asarray(logq_prop, dtype=f32)
    n = log_a.size
    u = np.array([_uniform24(seed, stream_base + c, DOMAIN_MH, rnd, 0, 0) for c in range(n)])
    with np.errstate(over="ignore", invalid="ignore"):
        e = np.exp(np.minimum(log_a.astype(np.float64), 0.0))
    accept = (log_a >= 0) | (u < np.exp(log_a.astype(f32)).astype(np.float64))
    ambiguous = (log_a < 0) & (np.abs(u - e) <= 4 * 2.0 ** -23 * e)
    return accept, ambiguous


DOMAIN_AUGMENT = 5


def augmented_minibatch(pool: np.ndarray, B: int, seed: int, stream_base: int, rnd: int):
    """Training minibatch under the symmetries of the periodic Boltzmann weight
    of Eq. (1) (global spin flip, translations): configuration b is pool
    member k under flip f and shift (di, dj), drawn from the domain-5 block
    of stream stream_base + b at counter (round lo, round hi, 0), words
    (x0, x1, x2, x3): k = floor((x1 2^32 + x0) P / 2^64), f = x2 & 1,
    di = (x2 >> 1) mod L, dj = x3 mod L; out[b][i][j] = (-1)^f
    pool[k][(i + di) mod L][(j + dj) mod L]."""
    from . import philox4x32_10

    pool = np.asarray(pool, dtype=np.int8)
    P, L = pool.shape[0], pool.shape[1]
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    out = np.empty((B, L, L), dtype=np.int8)
    for b in range(B):
        x = philox4x32_10((((stream_base + b) << 8) | (DOMAIN_AUGMENT << 4), rnd & 0xFFFFFFFF,
                           (rnd >> 32) & 0xFFFFFFFF, 0), key)
        k = (((x[1] << 32) | x[0]) * P) >> 64
        di, dj = (x[2] >> 1) % L, x[3] % L
        y = np.roll(pool[k], shift=(-di, -dj), axis=(0, 1))
        out[b] = -y if x[2] & 1 else y
    return out


def sample(theta, C: int, L: int, B: int, rng, emulate_bf16: bool = True):
    """Ancestral sampling site by site in raster order; returns (x, log q_exact)."""
    x = np.zeros((B, L, L))
    logq = np.zeros(B)
    for i in range(L):
        for j in range(L):
            logit, _ = forward(x, theta, C, emulate_bf16)
            Pq = quantised_p(logit[:, i, j])
            u = rng.integers(0, 1 << 24, B) / 2.0 ** 24
            up = u < Pq
            x[:, i, j] = np.where(up, 1.0, -1.0)
            with np.errstate(divide="ignore"):
                logq += np.where(up, np.log(Pq), np.log1p(-Pq))
    return x, logq
