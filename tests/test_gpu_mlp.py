"""GPU kernels of the learned flip proposal against the FP64 oracle:
forward logits, the BCE gradient, Adam training steps, determinism, and the
per-bit features of states (CPU oracle in oracle/mlp.py)."""
import numpy as np
import pytest

import oracle
import oracle.mlp as M
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2407_19987_amd import hobo

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return hobo, torch


def _dev(torch, a, dtype=None):
    import torch as T

    return T.from_numpy(np.ascontiguousarray(a, dtype=dtype or np.float32)).cuda()


def _params(seed):
    p = W.mlp_init(seed)
    rng = np.random.default_rng(seed + 1)
    p[M.OFF_B1:M.OFF_W2] = rng.normal(0, 0.3, M.HIDDEN)  # live and dead hidden units
    p[M.OFF_B2] = np.float32(-0.2)
    return p.astype(np.float32)


def _forward_scale(params, feats):
    """Sum of |terms| of each logit: the FP32 sums' error scale."""
    w1, b1, w2, b2 = M.unpack(M.rounded(params))
    f = np.asarray(feats, dtype=np.float64)
    pre = f @ w1 + b1
    preabs = np.abs(f) @ np.abs(w1) + np.abs(b1)
    return np.maximum(pre, 0) @ np.abs(w2) + preabs @ np.abs(w2) + abs(b2)


@pytest.mark.parametrize("m", [1, 1023, 5000])
def test_forward_matches_oracle(env, m):
    hobo, torch = env
    p = _params(1)
    f, _ = W.mlp_samples(m, seed=2)
    out = torch.empty(m, dtype=torch.float32, device="cuda")
    hobo.mlp_forward(_dev(torch, p), _dev(torch, f), out)
    got = out.cpu().numpy().astype(np.float64)
    want = M.forward(p, f)
    tol = 2e-5 * _forward_scale(p, f)  # 256-term FP32 sums: well under 2^-15 of the term scale
    assert (np.abs(got - want) <= tol).all()


@pytest.mark.parametrize("m", [1, 300, 4096, 9999])
def test_gradient_matches_oracle(env, m):
    hobo, torch = env
    p = _params(3)
    f, y = W.mlp_samples(m, seed=4)
    g = torch.empty(M.N_PARAM, dtype=torch.float32, device="cuda")
    ls = torch.empty(1, dtype=torch.float32, device="cuda")
    hobo.mlp_grad(_dev(torch, p), _dev(torch, f), _dev(torch, y), g, ls)
    loss, want = M.loss_grads(p, f, y)
    got = g.cpu().numpy().astype(np.float64)
    # error scale of each gradient entry: the sum over samples of |term|
    w1, b1, w2, b2 = M.unpack(M.rounded(p))
    ff = f.astype(np.float64)
    pre = ff @ w1 + b1
    lg = np.maximum(pre, 0) @ w2 + b2
    dl = np.abs(M.sigmoid(lg) - y) / m + 1e-30
    h = np.maximum(pre, 0)
    act = (pre > 0) * np.abs(w2)[None, :]
    sc = M.pack(np.abs(ff).T @ (dl[:, None] * act), (dl[:, None] * act).sum(0), h.T @ dl, dl.sum())
    assert (np.abs(got - want) <= 1e-4 * sc + 1e-9).all()
    assert abs(float(ls.cpu()[0]) - loss) <= 1e-5 * max(loss, 1.0)


def test_training_matches_oracle_and_is_deterministic(env):
    hobo, torch = env
    p0 = _params(5)
    f, _ = W.mlp_samples(6000, seed=6)
    y = (f[:, 1] < 0.5 * f[:, 0]).astype(np.float32)
    batch, epochs, lr = 1024, 2, 2e-3
    steps = epochs * ((6000 + batch - 1) // batch)
    outs = []
    for _ in range(2):
        st = torch.zeros(hobo.MLP_STATE, dtype=torch.float32, device="cuda")
        st[:M.N_PARAM] = _dev(torch, p0)
        lt = torch.empty(steps, dtype=torch.float32, device="cuda")
        hobo.mlp_train(st, _dev(torch, f), _dev(torch, y), batch=batch, epochs=epochs, lr=lr, loss_trace=lt)
        outs.append((st.cpu().numpy().copy(), lt.cpu().numpy().copy()))
    np.testing.assert_array_equal(outs[0][0], outs[1][0])  # fixed summation order
    np.testing.assert_array_equal(outs[0][1], outs[1][1])
    pw, _, _, losses = M.train(p0, f, y, batch=batch, epochs=epochs, lr=lr)
    np.testing.assert_allclose(outs[0][1], losses, rtol=2e-4, atol=1e-6)
    got = outs[0][0][:M.N_PARAM].astype(np.float64)
    # Adam steps are about lr in size whatever the gradient, so a gradient that
    # is zero within rounding may step either way: allow a few such entries
    d = np.abs(got - pw)
    assert np.mean(d <= 1e-3 * lr * steps + 1e-6 * np.abs(pw)) > 0.99
    assert d.max() <= 2 * lr * steps + 1e-6
    assert losses[-1] < losses[0]


@pytest.mark.parametrize("integer", [True, False])
def test_features_and_labels(env, integer):
    hobo, torch = env
    terms = W.cfg_int3(seed=7, n=21) if integer else W.cfg_real3(seed=7, n=40)
    c = oracle.canonicalize(terms)
    t = hobo.Tensor.from_terms(terms)
    # sweep 3 of a 9-sweep 4.0 -> 0.5 schedule: the library computes beta itself
    n, B, T0, T1, sw, L = c.n_vars, 77, 4.0, 0.5, 3, 9
    beta = 1.0 / oracle.schedule(T0, T1, L)[sw]
    x = W.random_states(n, B, seed=8)
    xa = W.random_states(n, B, seed=9)
    xb, xab = hobo.bits_to_device(W.pack_bits(x)), hobo.bits_to_device(W.pack_bits(xa))
    de = torch.empty((B, n), dtype=torch.int64 if integer else torch.float32, device="cuda")
    hobo.local_fields(t, xb, B, hobo.PREC_FP32, de)
    feats = torch.empty((B, n, 3), dtype=torch.float32, device="cuda")
    labels = torch.empty((B, n), dtype=torch.float32, device="cuda")
    hobo.proposal_features(t, xb, B, de, feats, t_start=T0, t_end=T1, sweep=sw, schedule_sweeps=L, x_after=xab,
                           labels_out=labels)
    got = feats.cpu().numpy()
    want = M.features(c, W.pack_bits(x), beta)
    np.testing.assert_array_equal(labels.cpu().numpy(), (x != xa).astype(np.float32))
    np.testing.assert_array_equal(got[..., 0], want[..., 0].astype(np.float32))
    np.testing.assert_array_equal(got[..., 2], want[..., 2].astype(np.float32))
    if integer:
        np.testing.assert_array_equal(got[..., 1], want[..., 1].astype(np.float32))
    else:
        sc = beta * oracle.field_scale(c, W.pack_bits(x))
        assert (np.abs(got[..., 1] - want[..., 1]) <= 1e-5 * np.maximum(np.abs(want[..., 1]), sc)).all()


def test_record_transitions_match_oracle_chain(env):
    """hobo_record_transitions on an integer instance: for each recorded sweep
    the features equal the oracle's features of the oracle chain's states at
    the start of that sweep (with that sweep's beta), and the labels its
    flips during the sweep."""
    hobo, torch = env
    terms = W.cfg_int3(seed=9, n=24)
    c = oracle.canonicalize(terms)
    t = hobo.Tensor.from_terms(terms)
    n, B, S, T0, T1, seed = c.n_vars, 40, 12, 4.0, 0.3, 21
    rec = [0, 3, 7, 11]
    feats = torch.empty((len(rec), B, n, 3), dtype=torch.float32, device="cuda")
    labels = torch.empty((len(rec), B, n), dtype=torch.float32, device="cuda")
    hobo.record_transitions(t, B, rec, feats, labels, sweeps=S, t_start=T0, t_end=T1, seed=seed,
                            precision=hobo.PREC_FP32)
    torch.cuda.synchronize()
    temps = oracle.schedule(T0, T1, S)
    x = oracle.anneal(c, B, 0, T0, T1, seed=seed)["final_bits"]  # the random start states
    s = 0
    for k, r in enumerate(rec):
        if r > s:
            x = oracle.anneal(c, B, r - s, T0, T1, seed=seed, init_bits=x, first_sweep=s, schedule_sweeps=S)["final_bits"]
        after = oracle.anneal(c, B, 1, T0, T1, seed=seed, init_bits=x, first_sweep=r, schedule_sweeps=S)["final_bits"]
        want = M.features(c, x, 1.0 / temps[r])
        np.testing.assert_array_equal(feats[k].cpu().numpy(), want.astype(np.float32))
        np.testing.assert_array_equal(labels[k].cpu().numpy(),
                                      (W.unpack_bits(x, n) != W.unpack_bits(after, n)).astype(np.float32))
        x, s = after, r + 1
