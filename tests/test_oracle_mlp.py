"""Pins for the oracle of the flip-proposal network (CPU only): BF16
rounding against torch's bfloat16 conversion, the loss against its closed
form, gradients against central finite differences and against autograd,
Adam against torch.optim.Adam, and the proposal rule's special cases."""
import math

import numpy as np
import pytest

import oracle
import oracle.mlp as M
import workloads as W


def test_bf16_round_ties_to_even_and_matches_torch():
    import torch

    one = 1.0
    cases = np.array([one, one + 2 ** -8, one + 3 * 2 ** -8, -2.5, 3.14159265, 1e-30, 65504.0, -7.0e-3],
                     dtype=np.float32)
    got = M.bf16_round(cases)
    assert got[0] == 1.0
    assert got[1] == 1.0  # exact tie, even neighbour is 1.0
    assert got[2] == np.float32(one + 2 ** -6)  # tie, even neighbour is 1 + 2^-6
    rng = np.random.default_rng(0)
    many = np.concatenate([cases, rng.normal(0, 10, 5000).astype(np.float32)])
    want = torch.from_numpy(many).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(M.bf16_round(many), want)


def test_loss_closed_form_at_zero_weights():
    f, y = W.mlp_samples(257, seed=1)
    p = np.zeros(M.N_PARAM)
    assert M.loss_raw(p, f, y) == pytest.approx(math.log(2.0), rel=1e-15)
    p[M.OFF_B2] = 0.75
    want = np.mean(np.log1p(np.exp(0.75)) - y.astype(np.float64) * 0.75)
    assert M.loss_raw(p, f, y) == pytest.approx(want, rel=1e-14)
    # with W1 = 0 the hidden layer is relu(b1): closed-form gradient of b2 and W2
    p[M.OFF_B1:M.OFF_W2] = np.linspace(-1, 1, M.HIDDEN)
    p[M.OFF_W2:M.OFF_B2] = 0.01
    _, g = M.loss_grads_raw(p, f, y)
    h = np.maximum(p[M.OFF_B1:M.OFF_W2], 0)
    l = h @ p[M.OFF_W2:M.OFF_B2] + 0.75
    dl = (1 / (1 + math.exp(-l)) - y.astype(np.float64)).mean()
    assert g[M.OFF_B2] == pytest.approx(dl, rel=1e-12)
    np.testing.assert_allclose(g[M.OFF_W2:M.OFF_B2], dl * h, rtol=1e-12, atol=1e-15)


def test_gradients_match_finite_differences():
    f, y = W.mlp_samples(64, seed=2)
    p = M.rounded(W.mlp_init(3) + np.float32(0.01))
    _, g = M.loss_grads_raw(p, f, y)
    rng = np.random.default_rng(4)
    for k in list(rng.choice(M.N_PARAM, 40, replace=False)) + [M.OFF_B2, M.OFF_W1, M.OFF_W2]:
        h = 1e-6
        a, b = p.copy(), p.copy()
        a[k] += h
        b[k] -= h
        fd = (M.loss_raw(a, f, y) - M.loss_raw(b, f, y)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(abs(g[k]), 1e-4), k


def test_gradients_match_autograd():
    import torch

    f, y = W.mlp_samples(300, seed=5)
    p = W.mlp_init(6)
    p[M.OFF_B1:M.OFF_W2] = 0.05
    loss, g = M.loss_grads(p, f, y)
    r = torch.tensor(M.rounded(p), dtype=torch.float64, requires_grad=True)
    w1 = r[M.OFF_W1:M.OFF_B1].reshape(3, 256)
    pre = torch.tensor(f, dtype=torch.float64) @ w1 + r[M.OFF_B1:M.OFF_W2]
    l = torch.relu(pre) @ r[M.OFF_W2:M.OFF_B2] + r[M.OFF_B2]
    lt = torch.nn.functional.binary_cross_entropy_with_logits(l, torch.tensor(y, dtype=torch.float64))
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-13)
    np.testing.assert_allclose(g, r.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_adam_matches_torch_and_first_step_is_signed_lr():
    import torch

    rng = np.random.default_rng(7)
    p0 = rng.normal(size=50)
    grads = [rng.normal(size=50) for _ in range(5)]
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    p1, _, _ = M.adam_step(p, grads[0], m, v, 1, lr=1e-3)
    np.testing.assert_allclose(p1 - p0, -1e-3 * grads[0] / (np.abs(grads[0]) + 1e-8), rtol=1e-12)
    tp = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t, g in enumerate(grads, 1):
        p, m, v = M.adam_step(p, g, m, v, t, lr=1e-3)
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_training_learns_a_threshold_rule():
    """Labels are 1 exactly when beta*dE < 0: a few epochs drive the loss far
    below the entropy of the labels."""
    f, _ = W.mlp_samples(4096, seed=8)
    y = (f[:, 1] < 0).astype(np.float32)
    p0 = W.mlp_init(9)
    p, _, _, losses = M.train(p0, f, y, batch=512, epochs=6, lr=3e-3)
    assert losses[0] > 0.4 and losses[-1] < 0.1
    assert np.asarray(p, dtype=np.float32).dtype == np.float32


def test_proposal_mask_special_cases():
    rng = np.random.default_rng(10)
    lg = rng.normal(size=(40, 20))
    sweeps = [3, 4]
    assert M.proposal_mask(lg, sweeps, tau=0.0, p_floor=0.0, seed=1).all()
    assert not M.proposal_mask(lg, sweeps, tau=1.0, p_floor=0.0, seed=1).any()
    assert M.proposal_mask(lg, sweeps, tau=1.0, p_floor=1.0, seed=1).all()
    m = M.proposal_mask(lg, sweeps, tau=0.5, p_floor=0.0, seed=1)
    want = np.stack([lg[16 * t:16 * t + 16].max(axis=0) >= 0.0 for t in range(3)])
    np.testing.assert_array_equal(m[:, 0], want)
    np.testing.assert_array_equal(m[:, 1], want)
    # floor draws are the Philox uniforms of counter (tile, sweep, i/4, 2)
    big = M.proposal_mask(np.full((16 * 8, 64), -50.0), list(range(16)), tau=0.5, p_floor=0.25, seed=3)
    assert abs(big.mean() - 0.25) < 0.02
    u = float(int(oracle.philox4x64([2, 5, 3, 2], [3, 0])[1]) >> 11) * 2.0 ** -53
    assert big[2, 5, 13] == (1 if u < 0.25 else 0)


def test_features_and_row_norms():
    terms = W.cfg_int3(seed=2, n=10)
    c = oracle.canonicalize(terms)
    rn = M.row_norms(c)
    # sum_i ||H_i||^2 counts every squared weight once per variable of its monomial
    assert np.sum(rn ** 2) == pytest.approx(sum(len(s) * float(w) ** 2 for s, w in zip(c.monos, c.weights)))
    x = W.random_states(10, 7, seed=3)
    bits = W.pack_bits(x)
    ft = M.features(c, bits, beta=0.5)
    np.testing.assert_array_equal(ft[..., 0], x)
    for b in range(7):
        for i in range(10):
            y = x[b].copy()
            y[i] ^= 1
            de = oracle.energy(c, W.pack_bits(y[None]))[0] - oracle.energy(c, W.pack_bits(x[b][None]))[0]
            assert ft[b, i, 1] == 0.5 * de
    np.testing.assert_allclose(ft[0, :, 2], 0.5 * rn)
