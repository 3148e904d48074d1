"""The symbolic front-end (expressions, integer encoding, compile with unused
symbols dropped) and the result aggregation, on the CPU.  The compiled
tensors of the paper's three worked problems (Sec. V), formulated through
the front-end from their statements, must equal the oracle's canonical form
of independently built term lists (multilinear expansions of each cost over
all states), reproduce the printed offsets 0 / 30 / 360 and, by brute force,
the printed minima -17 / -30 / -360 with every printed optimum among the
minimisers."""
import itertools

import numpy as np
import pytest

import oracle
import workloads as W
from paper_2407_19987_amd import frontend as F
from paper_2407_19987_amd import hobo


def _canon_of_compiled(cp):
    ptr, idx, w = cp.tensor.monomials()
    monos = [tuple(int(v) for v in idx[ptr[m]:ptr[m + 1]]) for m in range(len(w))]
    return sorted(zip(monos, [int(v) if cp.tensor.integer else float(v) for v in w]))


def _same_as(cp, terms):
    c = oracle.canonicalize(terms)
    assert _canon_of_compiled(cp) == sorted(zip(c.monos, c.weights))
    assert cp.offset == c.offset
    return c


def test_poly_algebra():
    x, y = F.symbol("ax"), F.symbol("ay")
    assert (x * x).t == x.t                      # x^2 = x for binary x
    assert ((1 - x) * x).t == {}                 # x (1 - x) = 0
    assert ((x + y) ** 2).t == (x + y + 2 * x * y).t
    assert (x - x).t == {} and (3 + x - 3).t == x.t
    v = F.int_var(3, "av{}")                     # 1 v0 + 2 v1 + 4 v2
    for m in range(8):
        assign = {F._NAMES.index(f"av{k}"): (m >> k) & 1 for k in range(3)}
        assert v.value(assign) == m
    a = F.symbols_list([2, 3], "aq{}_{}")
    assert a.shape == (2, 3) and F._NAMES[a[1, 2].symbols()[0]] == "aq1_2"
    p = np.prod(1 - a[0, :])                    # numpy reductions over symbol arrays
    assert p.value({}) == 1 and p.order == 3


def _seating_expr():
    q = F.symbols_list([5, 5], "q{}_{}")
    cells = [(i, j) for i in range(5) for j in range(5)]
    windows = [[(i, j + d) for d in range(3)] for i in range(5) for j in range(3)]
    windows += [[(i + d, j) for d in range(3)] for j in range(5) for i in range(3)]
    reward = sum(q[c] for c in cells)
    crowded = sum(q[w[0]] * q[w[1]] * q[w[2]] for w in windows)
    return q, 10 * crowded - reward


def _pythagorean_expr():
    q = F.symbols_list([3, 4], "p{}_{}")
    ints = [sum((1 << k) * q[p, k] for k in range(4)) for p in range(3)]
    zero = [np.prod(1 - q[p, :]) for p in range(3)]   # 1 iff integer p is 0
    return q, ints, (ints[0] ** 2 + ints[1] ** 2 - ints[2] ** 2) ** 2 + 10 * sum(zero)


def _tsp_expr():
    q = F.symbols_list([4, 2], "t{}_{}")     # a fourth integer is declared but not used
    ints = [2 * q[p, 0] + q[p, 1] for p in range(3)]
    return q, ints, 10 * (ints[0] * ints[1] * ints[2] - 6) ** 2


def test_seating_compiles_to_the_paper_instance(golden):
    q, h = _seating_expr()
    cp = F.compile_hobo(h)
    assert cp.n_vars == 25 and cp.offset == golden["seating"]["offset"] == 0
    c = _same_as(cp, W.paper_seating())
    best, n_min, args = oracle.brute_force(c, cap=64)
    assert best == golden["seating"]["min_energy"] == -17
    found = {tuple((a >> i) & 1 for i in range(25)) for a in args}
    for grid in golden["seating"]["printed_optima_grids"]:
        assert tuple(np.array(grid).reshape(-1)) in found


def test_pythagorean_compiles_to_the_paper_instance(golden):
    q, ints, h = _pythagorean_expr()
    cp = F.compile_hobo(h)
    assert cp.n_vars == 12 and cp.offset == golden["pythagorean"]["offset"] == 30
    c = _same_as(cp, W.paper_pythagorean())
    best, n_min, args = oracle.brute_force(c, cap=64)
    assert best == golden["pythagorean"]["min_energy"] == -30
    sol = set()
    for a in args:
        assign = {s: (a >> j) & 1 for j, s in enumerate(cp.symbol_ids)}
        sol.add(tuple(v.value(assign) for v in ints))
    assert {tuple(t) for t in golden["pythagorean"]["printed_optima_xyz"]} <= sol
    assert len(sol) == golden["pythagorean"]["n_solutions_text"] == 8


def test_tsp_compiles_with_unused_integer_dropped(golden):
    q, ints, h = _tsp_expr()
    cp = F.compile_hobo(h)
    # eight symbols declared, the six used ones kept (Sec. IV.D), in declaration order
    assert cp.n_vars == 6 and cp.names == ["t0_0", "t0_1", "t1_0", "t1_1", "t2_0", "t2_1"]
    assert cp.offset == golden["tsp_intenc"]["offset"] == 360
    c = _same_as(cp, W.paper_tsp_intenc())
    dense = cp.tensor.export_dense()
    assert list(dense.shape) == golden["tsp_intenc"]["tensor_shape"] and np.count_nonzero(dense) == 27
    best, n_min, args = oracle.brute_force(c, cap=64)
    assert best == golden["tsp_intenc"]["min_energy"] == -360
    sol = set()
    for a in args:
        assign = {s: (a >> j) & 1 for j, s in enumerate(cp.symbol_ids)}
        sol.add(tuple(v.value(assign) for v in ints))
    assert {tuple(t) for t in golden["tsp_intenc"]["printed_optima_BCD"]} <= sol
    assert sol == set(itertools.permutations((1, 2, 3)))


def test_compile_real_and_order_checks():
    x = F.symbols_list(3, "r{}")
    cp = F.compile_hobo(0.5 * x[0] * x[2] - 1.25 * x[1] + 2.0)
    assert not cp.tensor.integer and cp.offset == 2.0 and cp.n_vars == 3
    with pytest.raises(hobo.HoboError):
        F.compile_hobo(x[0] * x[1] * x[2], max_order=2)
    with pytest.raises(ValueError):
        F.compile_hobo(F.Poly({(): 3}))


def test_oracle_aggregate_by_hand():
    # four samples of two variables: states (1,0) twice, (0,1), (1,1)
    bits = np.array([[0b01, 0b10, 0b01, 0b11]], dtype=np.uint64)
    rows = oracle.aggregate(2, bits, [-1, -1, -1, 5])
    assert rows == [((0, 1), -1, 1, 1), ((1, 0), -1, 2, 0), ((1, 1), 5, 1, 3)]


@pytest.mark.parametrize("n,B,integer", [(7, 500, True), (70, 300, False), (130, 1000, True), (1, 9, True)])
def test_aggregate_matches_oracle(n, B, integer):
    """hobo_aggregate against the oracle's plain count: same states in the
    same order (energy, then bits), same first sample and count."""
    rng = np.random.default_rng(n + B)
    pool = W.random_states(n, 23, seed=n)                   # few distinct states, many repeats
    x = pool[rng.integers(0, 23, size=B)]
    bits = W.pack_bits(x)
    energy_of = {}
    for row in pool:
        energy_of.setdefault(tuple(row), int(rng.integers(-5, 5)) if integer else round(float(rng.normal()), 2))
    e = np.array([energy_of[tuple(r)] for r in x], dtype=np.int64 if integer else np.float64)
    rep, cnt = hobo.aggregate(n, bits, e)
    want = oracle.aggregate(n, bits, list(e))
    assert len(rep) == len(want) and int(cnt.sum()) == B
    for r, c, (_, _, cw, first) in zip(rep, cnt, want):
        assert int(r) == first and int(c) == cw
