"""Oracle of the learned flip proposal -- TEST INFRASTRUCTURE ONLY.

The paper names the stochastic search it runs over the HOBO tensor
(simulated annealing, Sec. II.D.1) and says nothing about a learned move
proposal; this module writes out, in FP64 numpy, the small network and the
proposal rule the engine adds on top of plain Metropolis, so that the GPU
kernels have a plain definition to be checked against:

* network   : a two-layer perceptron 3 -> 256 -> 1 over per-bit features,
              ``h = relu(W1^T f + b1)``, ``logit = W2 . h + b2``; the matrix
              weights enter the forward pass rounded to BF16 (round to
              nearest even), the biases in FP32;
* loss      : binary cross-entropy on the logit, ``softplus(l) - y l``,
              averaged over a minibatch;
* gradients : of that loss with respect to the (rounded) weights, applied to
              the FP32 master weights (straight-through rounding);
* optimiser : Adam (Kingma & Ba, ICLR 2015) with bias correction;
* features  : ``[x_i, beta dE_i, beta ||H_i||]`` for bit i of a state, with
              dE_i the single-flip change and ||H_i|| the Euclidean norm of
              all coefficients of monomials containing i;
* proposal  : a 16-replica tile attempts bit i during a segment iff some
              replica of the tile has ``logit >= logit(tau)`` or a floor draw
              u < p_floor (u from Philox4x64-10, counter (tile, sweep, i/4, 2),
              key (seed, instance), word i % 4, ``u = (r >> 11) 2^-53``).

Parameter vector layout (FP32, 1281 entries), shared with the GPU library:
``W1[f][u]`` at ``f*256+u`` (768), ``b1`` at 768, ``W2`` at 1024, ``b2`` at 1280.
"""
from __future__ import annotations

import math

import numpy as np

HIDDEN = 256
N_FEAT = 3
OFF_W1, OFF_B1, OFF_W2, OFF_B2 = 0, N_FEAT * HIDDEN, N_FEAT * HIDDEN + HIDDEN, N_FEAT * HIDDEN + 2 * HIDDEN
N_PARAM = OFF_B2 + 1


def bf16_round(a) -> np.ndarray:
    """Round FP32 values to the nearest BF16 value (ties to even), returned as
    FP32: keep the top 16 bits of the binary32 encoding after adding half an
    ulp of BF16 plus the parity of the kept part (finite inputs only)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    return (p[OFF_W1:OFF_B1].reshape(N_FEAT, HIDDEN), p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2], float(p[OFF_B2]))


def pack(w1, b1, w2, b2) -> np.ndarray:
    out = np.zeros(N_PARAM, dtype=np.float64)
    out[OFF_W1:OFF_B1] = np.asarray(w1, dtype=np.float64).reshape(-1)
    out[OFF_B1:OFF_W2] = b1
    out[OFF_W2:OFF_B2] = w2
    out[OFF_B2] = b2
    return out


def rounded(params) -> np.ndarray:
    """The weights the forward pass uses: W1, W2 rounded to BF16, biases as
    FP32 values (all returned in FP64)."""
    p32 = np.asarray(params, dtype=np.float32)
    out = p32.astype(np.float64)
    out[OFF_W1:OFF_B1] = bf16_round(p32[OFF_W1:OFF_B1])
    out[OFF_W2:OFF_B2] = bf16_round(p32[OFF_W2:OFF_B2])
    return out


def forward_raw(weights, feats):
    """Logits and pre-activations for the given weights, no rounding, FP64."""
    w1, b1, w2, b2 = unpack(weights)
    f = np.asarray(feats, dtype=np.float64).reshape(-1, N_FEAT)
    pre = f @ w1 + b1
    h = np.maximum(pre, 0.0)
    return h @ w2 + b2, pre


def forward(params, feats) -> np.ndarray:
    """Logits of the network with BF16-rounded matrix weights."""
    return forward_raw(rounded(params), feats)[0]


def softplus(x):
    x = np.asarray(x, dtype=np.float64)
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def sigmoid(x):
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(-np.abs(x))
    return np.where(x >= 0, 1.0 / (1.0 + e), e / (1.0 + e))


def loss_raw(weights, feats, labels) -> float:
    l, _ = forward_raw(weights, feats)
    y = np.asarray(labels, dtype=np.float64).reshape(-1)
    return float(np.mean(softplus(l) - y * l))


def loss_grads_raw(weights, feats, labels):
    """Mean BCE loss and its gradient (FP64, parameter-vector layout) at the
    given weights, by the chain rule through the two layers."""
    w1, b1, w2, b2 = unpack(weights)
    f = np.asarray(feats, dtype=np.float64).reshape(-1, N_FEAT)
    y = np.asarray(labels, dtype=np.float64).reshape(-1)
    m = len(y)
    pre = f @ w1 + b1
    h = np.maximum(pre, 0.0)
    l = h @ w2 + b2
    loss = float(np.mean(softplus(l) - y * l))
    dl = (sigmoid(l) - y) / m
    g_w2 = h.T @ dl
    g_b2 = float(np.sum(dl))
    dpre = np.outer(dl, w2) * (pre > 0.0)
    g_w1 = f.T @ dpre
    g_b1 = dpre.sum(axis=0)
    return loss, pack(g_w1, g_b1, g_w2, g_b2)


def loss_grads(params, feats, labels):
    """Loss and gradient of the network as the engine trains it: evaluated
    with the BF16-rounded weights, applied to the FP32 master weights."""
    return loss_grads_raw(rounded(params), feats, labels)


def adam_step(params, grads, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step number t >= 1); returns new (params, m, v)."""
    g = np.asarray(grads, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    p = np.asarray(params, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def train(params, feats, labels, batch: int, epochs: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
          eps: float = 1e-8, t0: int = 0, m=None, v=None):
    """Minibatch training in sample order (batch q holds samples
    [q*batch, (q+1)*batch), the last one possibly shorter), one Adam step per
    minibatch.  The master weights are kept in FP32 between steps, as on the
    GPU.  Returns (params, m, v, loss per step)."""
    f = np.asarray(feats, dtype=np.float64).reshape(-1, N_FEAT)
    y = np.asarray(labels, dtype=np.float64).reshape(-1)
    p = np.asarray(params, dtype=np.float32).astype(np.float64)
    m = np.zeros(N_PARAM) if m is None else np.asarray(m, dtype=np.float64)
    v = np.zeros(N_PARAM) if v is None else np.asarray(v, dtype=np.float64)
    t = t0
    losses = []
    for _ in range(epochs):
        for q0 in range(0, len(y), batch):
            loss, g = loss_grads(p, f[q0:q0 + batch], y[q0:q0 + batch])
            losses.append(loss)
            t += 1
            p, m, v = adam_step(p, g, m, v, t, lr, beta1, beta2, eps)
            p = p.astype(np.float32).astype(np.float64)
    return p, m, v, np.array(losses)


# ------------------------------------------------------------ proposal rule
def row_norms(canon) -> np.ndarray:
    """||H_i|| = sqrt(sum over monomials S containing i of w_S^2)."""
    out = np.zeros(canon.n_vars, dtype=np.float64)
    for mono, w in zip(canon.monos, canon.weights):
        for i in mono:
            out[i] += float(w) ** 2
    return np.sqrt(out)


def features(canon, bits, beta: float) -> np.ndarray:
    """[B][N][3] features of every bit of every row of ``bits`` ([W][B]
    words): x_i, beta * dE_i, beta * ||H_i||."""
    import oracle
    import workloads as W

    x = W.unpack_bits(np.asarray(bits, dtype=np.uint64), canon.n_vars)
    _, de = oracle.fields(canon, bits)
    out = np.zeros(x.shape + (3,), dtype=np.float64)
    out[..., 0] = x
    out[..., 1] = beta * np.asarray(de, dtype=np.float64)
    out[..., 2] = beta * row_norms(canon)[None, :]
    return out


def floor_uniform(tile: int, sweep: int, i: int, seed: int, inst: int = 0) -> float:
    import oracle

    r = oracle.philox4x64([tile, sweep, i // 4, 2], [seed, inst])[i % 4]
    return float(int(r) >> 11) * 2.0 ** -53


def proposal_mask(logits, sweeps, tau: float, p_floor: float, seed: int, inst: int = 0) -> np.ndarray:
    """Attempt masks [ceil(B/16)][len(sweeps)][N] from logits [B][N] taken at
    the segment start: tile t attempts bit i in sweep s iff
    max_{b in t} logit_{b,i} >= logit(tau) or u(t, s, i) < p_floor."""
    lg = np.asarray(logits, dtype=np.float64)
    b, n = lg.shape
    nt = (b + 15) // 16
    thr = math.log(tau / (1.0 - tau)) if 0.0 < tau < 1.0 else (-math.inf if tau <= 0.0 else math.inf)
    out = np.zeros((nt, len(sweeps), n), dtype=np.uint8)
    for t in range(nt):
        hot = lg[16 * t:16 * t + 16].max(axis=0) >= thr
        for k, s in enumerate(sweeps):
            for i in range(n):
                out[t, k, i] = 1 if hot[i] or floor_uniform(t, s, i, seed, inst) < p_floor else 0
    return out
