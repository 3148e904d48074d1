"""Gradient-descent search (Sec. II.D.2) on the GPU against the oracle
(oracle/gd.py): the gradient of the multilinear extension at random points,
the Philox start, whole runs of projected steps, the rounding and the exact
energies of the rounded states."""
import numpy as np
import pytest

import oracle
import oracle.gd as G
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2407_19987_amd import hobo

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return hobo, torch


def _inst(seed, n, k, integer, dens=0.6):
    rng = np.random.default_rng(seed)
    subs, co = [], []
    for r in range(1, k + 1):
        s = W.lex_subsets(n, r)
        keep = rng.random(len(s)) < (dens if n < 200 else 0.1)
        subs.append(s[keep])
        co.append(rng.integers(-6, 7, size=int(keep.sum())) if integer else
                  rng.standard_normal(int(keep.sum())).astype(np.float32).astype(np.float64))
    return W.subsets_to_terms(n, subs, co, integer)


CASES = [(1, 7, 3, False), (2, 37, 3, True), (3, 20, 4, False), (4, 130, 2, False), (5, 70, 3, False),
         (6, 256, 2, False), (7, 14, 6, True)]


@pytest.mark.parametrize("seed,n,k,integer", CASES)
def test_gradient_matches_oracle(env, seed, n, k, integer):
    hobo, torch = env
    terms = _inst(seed, n, k, integer)
    c = oracle.canonicalize(terms)
    t = hobo.Tensor.from_terms(terms)
    B = 77
    p = np.random.default_rng(seed).random((B, n))
    pd = torch.from_numpy(np.ascontiguousarray(p.T)).cuda()
    gd = torch.zeros_like(pd)
    hobo.gd_gradient(t, pd, B, gd)
    torch.cuda.synchronize()
    # the kernel forms each product over the other variables in index order
    # and adds the monomials in list order, rounding every operation
    # separately, as the oracle does: equal bit for bit
    np.testing.assert_array_equal(gd.cpu().numpy().T, G.gradient(c, p))


@pytest.mark.parametrize("seed,n,k,integer", CASES)
def test_descent_run_matches_oracle(env, seed, n, k, integer):
    """Random Philox start, 12 projected steps, rounding and exact energies,
    all equal to the oracle's bit for bit (every step's products, sums and
    p - eta g are rounded separately on both sides)."""
    hobo, torch = env
    terms = _inst(seed, n, k, integer)
    c = oracle.canonicalize(terms)
    t = hobo.Tensor.from_terms(terms)
    B, T = 50, 12
    eta = 0.5 / max(1.0, max(abs(float(w)) for w in c.weights) * n)
    p = torch.zeros(n * B, dtype=torch.float64, device="cuda")
    x = torch.zeros(((n + 63) // 64) * B, dtype=torch.int64, device="cuda")
    e = torch.zeros(B, dtype=torch.int64 if integer else torch.float64, device="cuda")
    hobo.gd_batch(t, B, p, x, e, iterations=0, eta=eta, seed=23)
    torch.cuda.synchronize()
    p0 = G.random_start(n, B, seed=23)
    np.testing.assert_array_equal(p.cpu().numpy().reshape(n, B).T, p0)
    hobo.gd_batch(t, B, p, x, e, iterations=T, eta=eta, seed=23, init=hobo.INIT_GIVEN)
    torch.cuda.synchronize()
    pT = G.descend(c, p0, T, eta)
    np.testing.assert_array_equal(p.cpu().numpy().reshape(n, B).T, pT)
    xg = W.unpack_bits(hobo.bits_to_host(x).reshape((n + 63) // 64, B), n)
    xo, _ = G.round_and_score(c, pT)
    np.testing.assert_array_equal(xg, xo)
    np.testing.assert_array_equal(e.cpu().numpy(), oracle.energy(c, W.pack_bits(xg)))


def test_descent_lowers_the_energy(env):
    """On an N=64 order-3 instance of the benchmark's distribution, 300 steps
    from 2048 random starts end in rounded states far below random states."""
    hobo, torch = env
    terms = W.cfg_real3(seed=8, n=64)
    t = hobo.Tensor.from_terms(terms)
    c = oracle.canonicalize(terms)
    B, n = 2048, 64
    p = torch.zeros(n * B, dtype=torch.float64, device="cuda")
    x = torch.zeros(B, dtype=torch.int64, device="cuda")
    e = torch.zeros(B, dtype=torch.float64, device="cuda")
    hobo.gd_batch(t, B, p, x, e, iterations=300, eta=0.05, seed=4)
    torch.cuda.synchronize()
    rand = oracle.energy(c, W.pack_bits(W.random_states(n, 256, seed=1)))
    got = e.cpu().numpy()
    assert np.median(got) < np.percentile(rand, 1)
    print(f"gradient descent: median {np.median(got):.4f}, best {got.min():.4f}; random states median "
          f"{np.median(rand):.4f}")
