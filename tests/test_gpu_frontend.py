"""The three worked problems of Sec. V end to end on the GPU: formulated
through the front-end, compiled, sampled with 10000 shots (the paper's
batch), and aggregated into the result list.  The best energy must be the
printed minimum, every printed optimum must be among the minimum-energy rows
(decoded back to seat grids and integers), and the occurrences must add up to
the shots; the row energies are the oracle's energies of the row states."""
import numpy as np
import pytest

import oracle
import workloads as W
from paper_2407_19987_amd import frontend as F

from test_frontend import _pythagorean_expr, _seating_expr, _tsp_expr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch


def _check_rows(rows, cp, shots, min_e):
    assert sum(r.occurrence for r in rows) == shots
    es = [r.energy for r in rows]
    assert es == sorted(es) and es[0] == min_e
    # row energies are the exact energies of the row states
    ptr, idx, w = cp.tensor.monomials()
    c = oracle.canonicalize(W.TermList(cp.n_vars, ptr, idx, w, "compiled"))
    x = np.array([r.bits for r in rows[:50]], dtype=np.uint8)
    np.testing.assert_array_equal(oracle.energy(c, W.pack_bits(x)), es[:50])
    return [r for r in rows if r.energy == min_e]


def test_seating_end_to_end(gpu, golden):
    q, h = _seating_expr()
    cp = F.compile_hobo(h)
    rows = F.sample(cp, 10000, sweeps=300, seed=1)
    best = _check_rows(rows, cp, 10000, golden["seating"]["min_energy"])
    grids = {tuple(r.array("q{}_{}")[0].reshape(-1)) for r in best}
    for g in golden["seating"]["printed_optima_grids"]:
        assert tuple(np.array(g).reshape(-1)) in grids


def test_pythagorean_end_to_end(gpu, golden):
    q, ints, h = _pythagorean_expr()
    cp = F.compile_hobo(h)
    rows = F.sample(cp, 10000, sweeps=300, seed=2)
    best = _check_rows(rows, cp, 10000, golden["pythagorean"]["min_energy"])
    sol = {tuple(r.value(v) for v in ints) for r in best}
    assert {tuple(t) for t in golden["pythagorean"]["printed_optima_xyz"]} <= sol


def test_tsp_end_to_end(gpu, golden):
    q, ints, h = _tsp_expr()
    cp = F.compile_hobo(h)
    rows = F.sample(cp, 10000, sweeps=300, seed=3)
    best = _check_rows(rows, cp, 10000, golden["tsp_intenc"]["min_energy"])
    sol = {tuple(r.value(v) for v in ints) for r in best}
    assert {tuple(t) for t in golden["tsp_intenc"]["printed_optima_BCD"]} <= sol
