"""hobo_autotune picks launch shapes by timing; results never depend on the
shape: energies, flip changes and annealing trajectories after tuning equal
those before, bit for bit, and equal the oracle's on integer instances."""
import numpy as np
import pytest

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_keeps_results(env_tune=None):
    import torch

    from paper_2407_19987_amd import hobo

    assert torch.cuda.is_available()
    terms = W.cfg_int3(seed=21, n=40)
    c = oracle.canonicalize(terms)
    t = hobo.Tensor.from_terms(terms)
    B = 700
    bits = W.pack_bits(W.random_states(40, B, seed=22))
    xb = hobo.bits_to_device(bits)

    def run():
        e = torch.zeros(B, dtype=torch.int64, device="cuda")
        de = torch.zeros((B, 40), dtype=torch.int64, device="cuda")
        hobo.energy(t, xb, B, hobo.PREC_BF16X2, e)
        hobo.local_fields(t, xb, B, hobo.PREC_BF16X2, de)
        x = xb.clone()
        bx = torch.zeros_like(x)
        be = torch.zeros(B, dtype=torch.int64, device="cuda")
        hobo.anneal_batch(t, B, x, bx, be, sweeps=30, t_start=3.0, t_end=0.1, seed=5, precision=hobo.PREC_BF16X2,
                          init=hobo.INIT_GIVEN)
        torch.cuda.synchronize()
        return e.cpu().numpy(), de.cpu().numpy(), hobo.bits_to_host(bx), be.cpu().numpy()

    before = run()
    shapes = hobo.autotune(t, xb, B, 7, hobo.PREC_BF16X2)
    assert shapes[0] in {16 * r + c for r in (1, 2, 4) for c in (1, 2, 4, 8)}
    assert shapes[1] in {16 * r + c for r in (1, 2, 4) for c in (1, 2, 4, 8)}
    assert shapes[2] in (1, 2, 4, 8)
    after = run()
    for a, b in zip(before, after):
        np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(after[0], oracle.energy(c, bits))
    np.testing.assert_array_equal(after[1], oracle.fields(c, bits)[1])
    o = oracle.anneal(c, B, 30, 3.0, 0.1, seed=5, init_bits=bits)
    np.testing.assert_array_equal(after[3], o["best_e"])
