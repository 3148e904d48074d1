"""Oracle for the gradient-descent search (Sec. II.D.2).

Test infrastructure, like the rest of oracle/: only the tests, the smoke
entry point and the benchmark's CPU-baseline leg use it.

The paper names gradient descent on the cost, with variables updated along
the gradient and mini-batch variants, and fixes nothing else.  The reading
implemented (and listed with the others in the design notes):

* the cost of a continuous point p in [0, 1]^N is the multilinear extension
  E(p) = sum_S w_S prod_{i in S} p_i, which equals the HOBO energy at every
  binary point;
* its gradient is g_i(p) = dE/dp_i = sum_{S containing i} w_S prod_{j in S, j != i} p_j
  (at a binary point, the local field of bit i);
* one step moves every coordinate against the gradient and projects back
  onto the box: p <- min(1, max(0, p - eta g(p))), all coordinates of a
  replica from the same p (a full-gradient step); a batch of replicas runs
  independently (the mini-batch of starting points);
* the random start draws p_i = (r >> 11) 2^-53 from Philox4x64-10 word i % 4
  at counter (replica, 0, i / 4, 3), key (seed, 0);
* the answer is the rounded point x_i = [p_i > 1/2], judged by its exact
  energy.
"""
from __future__ import annotations

import numpy as np

from . import Canonical, energy as _energy, philox4x64


def gradient(canon: Canonical, p: np.ndarray) -> np.ndarray:
    """g[b, i] = sum over monomials S containing i of w_S prod_{j in S - i} p[b, j]."""
    p = np.asarray(p, dtype=np.float64)
    g = np.zeros_like(p)
    for mono, w in zip(canon.monos, canon.weights):
        for i in mono:
            prod = np.full(p.shape[0], float(w))
            for j in mono:
                if j != i:
                    prod = prod * p[:, j]
            g[:, i] += prod
    return g


def extension(canon: Canonical, p: np.ndarray) -> np.ndarray:
    """E(p) = sum_S w_S prod_{i in S} p_i for each row of p."""
    p = np.asarray(p, dtype=np.float64)
    e = np.zeros(p.shape[0])
    for mono, w in zip(canon.monos, canon.weights):
        prod = np.full(p.shape[0], float(w))
        for i in mono:
            prod = prod * p[:, i]
        e += prod
    return e


def random_start(n_vars: int, n_rep: int, seed: int) -> np.ndarray:
    """p[b, i] from Philox4x64-10 word i % 4 at counter (b, 0, i // 4, 3), key (seed, 0)."""
    p = np.zeros((n_rep, n_vars))
    for b in range(n_rep):
        for q in range((n_vars + 3) // 4):
            words = philox4x64(np.array([b, 0, q, 3], dtype=np.uint64), (seed, 0))
            for e in range(4):
                i = 4 * q + e
                if i < n_vars:
                    p[b, i] = (int(words[e]) >> 11) * 2.0 ** -53
    return p


def descend(canon: Canonical, p0: np.ndarray, iterations: int, eta: float) -> np.ndarray:
    """Projected full-gradient steps p <- clip(p - eta g(p), 0, 1)."""
    p = np.array(p0, dtype=np.float64)
    for _ in range(iterations):
        p = np.clip(p - eta * gradient(canon, p), 0.0, 1.0)
    return p


def round_and_score(canon: Canonical, p: np.ndarray):
    """x = [p > 1/2] as [B][N] uint8 and its exact energies."""
    x = (np.asarray(p) > 0.5).astype(np.uint8)
    n = canon.n_vars
    w = (n + 63) // 64
    bits = np.zeros((w, x.shape[0]), dtype=np.uint64)
    for i in range(n):
        bits[i >> 6] |= x[:, i].astype(np.uint64) << np.uint64(i & 63)
    return x, _energy(canon, bits)
