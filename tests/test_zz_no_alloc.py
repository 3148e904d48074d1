"""hobo_energy_noalloc (the energy entry point that allocates nothing and
works in the library's per-GPU scratch) against hobo_energy: identical
results on two calls in a row, the second with a smaller batch, for every
precision family; clear refusals when the layout is not prepared or the batch
needs more scratch than there is."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    from paper_2407_19987_amd import hobo

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return hobo, torch


CASES = [("real3", lambda: W.cfg_real3(seed=6), 5), ("real3", lambda: W.cfg_real3(seed=6), 0),
         ("real3", lambda: W.cfg_real3(seed=6), 4), ("intenc4", lambda: W.cfg_intenc4(seed=1), 3),
         ("int3", lambda: W.cfg_int3(seed=5, n=40), 1)]


@pytest.mark.parametrize("name,make,prec", CASES)
def test_noalloc_matches_energy_twice(env, name, make, prec):
    hobo, torch = env
    t = hobo.Tensor.from_terms(make())
    t.prepare(hobo.FN_ENERGY, 1 << prec)
    dt = torch.int64 if t.integer else torch.float64
    for B, seed in ((4096, 1), (777, 2)):
        xb = hobo.bits_to_device(W.pack_bits(W.random_states(t.n_vars, B, seed=seed)))
        want = torch.zeros(B, dtype=dt, device="cuda")
        hobo.energy(t, xb, B, prec, want)
        got = torch.full((B,), 7, dtype=dt, device="cuda")
        hobo.energy_noalloc(t, xb, B, prec, got)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got.cpu().numpy(), want.cpu().numpy())


def test_noalloc_refusals_and_empty(env):
    hobo, torch = env
    t = hobo.Tensor.from_terms(W.cfg_real3(seed=7, n=64))
    xb = hobo.bits_to_device(W.pack_bits(W.random_states(64, 100, seed=3)))
    e = torch.zeros(100, dtype=torch.float64, device="cuda")
    with pytest.raises(hobo.HoboError) as ei:  # layout not prepared
        hobo.energy_noalloc(t, xb, 100, hobo.PREC_BF16X2, e)
    assert ei.value.code == hobo.ERR_INVALID_ARG
    t.prepare(hobo.FN_ENERGY, 1 << hobo.PREC_BF16X2)
    hobo.energy_noalloc(t, xb, 100, hobo.PREC_BF16X2, e)
    # a batch whose workspace exceeds the 32 MiB scratch is refused before any
    # launch (FP64: 11 groups of 4096 monomials x 8 B per replica)
    t.prepare(hobo.FN_ENERGY, 1 << hobo.PREC_FP64)
    big = 1 << 20
    xbig = torch.zeros(big, dtype=torch.int64, device="cuda")
    ebig = torch.zeros(big, dtype=torch.float64, device="cuda")
    with pytest.raises(hobo.HoboError) as ei:
        hobo.energy_noalloc(t, xbig, big, hobo.PREC_FP64, ebig)
    assert ei.value.code == hobo.ERR_INVALID_ARG
    # no monomials: the energies are zero-filled
    t0 = hobo.Tensor.from_terms(W.poly_to_terms(5, W.RawPoly.const(3.5), False))
    x0 = hobo.bits_to_device(W.pack_bits(W.random_states(5, 50, seed=1)))
    e0 = torch.full((50,), 9.0, dtype=torch.float64, device="cuda")
    hobo.energy_noalloc(t0, x0, 50, hobo.PREC_FP32, e0)
    torch.cuda.synchronize()
    assert (e0.cpu().numpy() == 0.0).all()
