"""Pins for the CPU oracle: what the paper prints and what the mathematics
fixes, independent of the oracle's own code paths (CPU only)."""
import itertools
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _canon(t):
    return oracle.canonicalize(t)


# ---------------------------------------------------------------- paper pins


def test_seating_problem_pins(golden):
    g = golden["seating"]
    c = _canon(W.paper_seating())
    assert c.n_vars == 25 and c.order == 3
    assert c.offset == g["offset"]
    best, nmin, args = oracle.brute_force(c)
    assert best == g["min_energy"]
    found = {a for a in args}
    for grid in g["printed_optima_grids"]:
        x = np.array(grid, dtype=np.uint8).reshape(-1)
        code = int(sum(int(v) << i for i, v in enumerate(x)))
        assert code in found
        e = oracle.energy(c, W.pack_bits(x[None, :]))
        assert int(e[0]) == g["min_energy"]


def test_pythagorean_problem_pins(golden):
    g = golden["pythagorean"]
    c = _canon(W.paper_pythagorean())
    assert c.n_vars == 12 and c.order == 4
    assert c.offset == g["offset"]
    best, nmin, args = oracle.brute_force(c)
    assert best == g["min_energy"]
    assert nmin == g["n_solutions_text"]
    sols = set()
    for a in args:
        row = np.array([(a >> i) & 1 for i in range(12)], dtype=np.uint8)
        sols.add(tuple(W.decode_int(row, 4 * p, 4) for p in range(3)))
    for xyz in g["printed_optima_xyz"]:
        assert tuple(xyz) in sols
    # every minimiser is a Pythagorean triple with positive entries
    for x, y, z in sols:
        assert x * x + y * y == z * z and min(x, y, z) > 0


def test_tsp_problem_pins(golden):
    g = golden["tsp_intenc"]
    c = _canon(W.paper_tsp_intenc())
    assert c.n_vars == 6 and c.order == 6
    assert c.offset == g["offset"]
    best, nmin, args = oracle.brute_force(c)
    assert best == g["min_energy"]
    sols = set()
    for a in args:
        row = np.array([(a >> i) & 1 for i in range(6)], dtype=np.uint8)
        sols.add(tuple(W.decode_int(row, 2 * p, 2, msb_first=True) for p in range(3)))
    assert sols == set(itertools.permutations((1, 2, 3)))
    for bcd in g["printed_optima_BCD"]:
        assert tuple(bcd) in sols


def test_tsp_tensor_layout_and_tt_ranks(golden):
    """Sec. VI.F: the order-6 tensor is (6,)^6 and its exact TT decomposition
    has the printed core shapes -- which holds for the smallest-index
    replication layout of Sec. III.C in declaration order."""
    g = golden["tsp_intenc"]
    c = _canon(W.paper_tsp_intenc())
    h = oracle.paper_tensor(c)
    assert list(h.shape) == g["tensor_shape"]
    assert np.count_nonzero(h) == len(c.monos) == 27
    n, d = 6, 6
    ranks = [int(np.linalg.matrix_rank(h.reshape(n ** j, n ** (d - j)).astype(np.float64))) for j in range(1, d)]
    shapes = [[n, ranks[0]]] + [[ranks[j - 1], n, ranks[j]] for j in range(1, d - 1)] + [[ranks[-1], n]]
    assert shapes == g["tt_core_shapes"]


def test_tsp_einsum_path_counts(golden):
    """The dense-contraction cost the paper prints for the (6,)^6 tensor."""
    g = golden["tsp_intenc"]["einsum_dense"]
    c = _canon(W.paper_tsp_intenc())
    h = oracle.paper_tensor(c).astype(np.float64)
    x = np.ones(6)
    _, text = np.einsum_path("i,j,k,l,m,n,ijklmn->", x, x, x, x, x, x, h, optimize="greedy")
    assert f"{g['naive_flops']:.3e}" in text
    assert f"{g['optimized_flops']:.3e}" in text
    assert f"{g['largest_intermediate']:.3e}" in text


# ------------------------------------------------------- mathematical pins


def _rand_int_instance(seed, n, k, lo=-5, hi=5, dens=0.7):
    rng = np.random.default_rng(seed)
    subs, co = [], []
    for r in range(1, k + 1):
        s = W.lex_subsets(n, r)
        keep = rng.random(len(s)) < dens
        subs.append(s[keep])
        co.append(rng.integers(lo, hi + 1, size=int(keep.sum())))
    return W.subsets_to_terms(n, subs, co, True)


def _rand_real_instance(seed, n, k, dens=0.8):
    rng = np.random.default_rng(seed)
    subs, co = [], []
    for r in range(1, k + 1):
        s = W.lex_subsets(n, r)
        keep = rng.random(len(s)) < dens
        subs.append(s[keep])
        co.append(rng.standard_normal(int(keep.sum())).astype(np.float32).astype(np.float64))
    return W.subsets_to_terms(n, subs, co, False)


def test_canonical_form_rules():
    # x0*x0*x1 (repeat) + 2*x1*x0 (duplicate, other order) + 3 (constant) - 3*x0*x1 (cancels)
    p = W.RawPoly([((0, 0, 1), 1), ((1, 0), 2), ((), 3), ((0, 1), -3), ((2,), 5), ((2, 2), -5), ((), -1)])
    c = oracle.canonicalize(W.poly_to_terms(3, p, True))
    assert c.monos == [] and c.offset == 2 and c.order == 0
    p = W.RawPoly([((3, 1, 1), 4), ((1, 3), 1), ((0,), -2)])
    c = oracle.canonicalize(W.poly_to_terms(4, p, True))
    assert c.monos == [(0,), (1, 3)] and c.weights == [-2, 5] and c.order == 2


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_matches_definition(seed):
    t = _rand_int_instance(seed, 10, 4)
    c = _canon(t)
    e = oracle.energy(c, W.pack_bits(W.all_states(10)))
    best, nmin, args = oracle.brute_force(c, cap=1024)
    assert best == int(e.min())
    assert nmin == int((e == e.min()).sum())
    assert sorted(args) == sorted(np.nonzero(e == e.min())[0].tolist())


def test_special_states():
    t = _rand_int_instance(7, 12, 3)
    c = _canon(t)
    n = c.n_vars
    x = np.zeros((n + 2, n), dtype=np.uint8)
    for i in range(n):
        x[i + 1, i] = 1
    x[n + 1, :] = 1
    e = oracle.energy(c, W.pack_bits(x))
    lin = {m[0]: w for m, w in zip(c.monos, c.weights) if len(m) == 1}
    assert e[0] == 0  # offset excluded
    for i in range(n):
        assert e[i + 1] == lin.get(i, 0)
    assert e[n + 1] == sum(c.weights)


def test_qubo_form():
    t = _rand_int_instance(3, 20, 2, dens=1.0)
    c = _canon(t)
    q = oracle.qubo_matrix(c)
    x = W.random_states(20, 300, seed=5)
    e = oracle.energy(c, W.pack_bits(x))
    ref = np.einsum("bi,ij,bj->b", x.astype(np.int64), q, x.astype(np.int64))
    np.testing.assert_array_equal(e, ref)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_paper_tensor_contraction_and_symmetrisation(k):
    """Contracting the paper-layout tensor with x k times gives E, and so does
    the symmetrised tensor (1/k!) sum over index permutations."""
    t = _rand_real_instance(11 + k, 7, k)
    c = _canon(t)
    h = oracle.paper_tensor(c)
    x = W.random_states(7, 40, seed=9)
    e = oracle.energy(c, W.pack_bits(x))
    np.testing.assert_allclose(oracle.tensor_contract(h, x), e, rtol=0, atol=1e-12)
    hs = sum(np.transpose(h, p) for p in itertools.permutations(range(k))) / math.factorial(k)
    np.testing.assert_allclose(oracle.tensor_contract(hs, x), e, rtol=0, atol=1e-12)
    # the upper-triangular replicated layout: every non-zero sits at a
    # non-decreasing index tuple whose leading run is the smallest index
    for idx in zip(*np.nonzero(h)):
        assert list(idx) == sorted(idx)


def test_real_energy_is_correctly_rounded():
    t = W.cfg_real3(seed=3, n=24)
    c = _canon(t)
    x = W.random_states(24, 50, seed=4)
    e = oracle.energy(c, W.pack_bits(x))
    for b in range(50):
        on = [w for m, w in zip(c.monos, c.weights) if all(x[b, i] for i in m)]
        assert e[b] == math.fsum(on)


@pytest.mark.parametrize("integer", [True, False])
def test_flip_changes_by_definition(integer):
    t = _rand_int_instance(5, 14, 4) if integer else _rand_real_instance(5, 14, 4)
    c = _canon(t)
    x = W.random_states(14, 64, seed=6)
    g, de = oracle.fields(c, W.pack_bits(x))
    e0 = oracle.energy(c, W.pack_bits(x))
    for i in range(14):
        xf = x.copy()
        xf[:, i] ^= 1
        e1 = oracle.energy(c, W.pack_bits(xf))
        if integer:
            np.testing.assert_array_equal(e1 - e0, de[:, i])
            np.testing.assert_array_equal(e1 - e0, (1 - 2 * x[:, i].astype(np.int64)) * g[:, i])
        else:
            np.testing.assert_allclose(e1 - e0, de[:, i], rtol=0, atol=1e-12)


def test_euler_identity_per_order():
    """sum_i x_i g_i^(r) = r E^(r) for the order-r part of an instance."""
    t = _rand_int_instance(8, 16, 4)
    c = _canon(t)
    x = W.random_states(16, 100, seed=2)
    bits = W.pack_bits(x)
    for r in range(1, 5):
        sub = oracle.Canonical(c.n_vars, r, [m for m in c.monos if len(m) == r],
                               [w for m, w in zip(c.monos, c.weights) if len(m) == r], 0, True)
        g, _ = oracle.fields(sub, bits)
        np.testing.assert_array_equal((x.astype(np.int64) * g).sum(axis=1), r * oracle.energy(sub, bits))


def test_minimisers_are_local_minima():
    c = _canon(W.paper_pythagorean())
    best, nmin, args = oracle.brute_force(c)
    x = np.array([[(a >> i) & 1 for i in range(12)] for a in args], dtype=np.uint8)
    _, de = oracle.fields(c, W.pack_bits(x))
    assert (de >= 0).all()


# ---------------------------------------------------------------- Philox


@pytest.mark.parametrize("ctr,key", [((0, 0, 0, 0), (0, 0)), ((5, 9, 1, 0), (12345, 3)),
                                     ((2 ** 64 - 1, 7, 2 ** 63, 1), (2 ** 64 - 1, 2 ** 40))])
def test_philox_known_answers(ctr, key):
    """numpy.random.Philox is Philox4x64-10; it increments the counter before
    each block, so start it one below the wanted counter."""
    c0 = list(ctr)
    start = np.array(c0, dtype=np.uint64)
    # subtract one with borrow across words
    words = [int(v) for v in c0]
    for j in range(4):
        if words[j] > 0:
            words[j] -= 1
            break
        words[j] = 2 ** 64 - 1
    ref = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(words, dtype=np.uint64))
    want = ref.random_raw(4)
    got = oracle.philox4x64(start, key)
    np.testing.assert_array_equal(got, want)


# ---------------------------------------------------------------- annealer


def test_metropolis_stationary_distribution():
    """At a fixed temperature the sequential single-flip Metropolis chain
    leaves the Boltzmann distribution invariant: after many sweeps the
    replicas' states follow exp(-E/T)/Z (chi-square over all 2^6 states)."""
    n, T = 6, 1.5
    c = _canon(_rand_real_instance(21, n, 3, dens=1.0))
    res = oracle.anneal(c, n_rep=6000, sweeps=60, t_start=T, t_end=T, seed=77)
    x = W.unpack_bits(res["final_bits"], n)
    codes = (x.astype(np.int64) << np.arange(n)).sum(axis=1)
    counts = np.bincount(codes, minlength=2 ** n)
    e = oracle.energy(c, W.pack_bits(W.all_states(n)))
    p = np.exp(-(e - e.min()) / T)
    p /= p.sum()
    expected = p * len(codes)
    mask = expected > 5
    chi2 = (((counts - expected) ** 2) / expected)[mask].sum()
    from scipy.stats import chi2 as chi2d

    assert chi2d.sf(chi2, int(mask.sum()) - 1) > 1e-4


def test_anneal_reaches_paper_minima(golden):
    for f, key in ((W.paper_seating, "seating"), (W.paper_pythagorean, "pythagorean"), (W.paper_tsp_intenc, "tsp_intenc")):
        c = _canon(f())
        res = oracle.anneal(c, n_rep=256, sweeps=200, t_start=5.0, t_end=0.05, seed=1)
        assert int(res["best_e"].min()) == golden[key]["min_energy"]
        # best energies are exact energies of the best states
        np.testing.assert_array_equal(res["best_e"], oracle.energy(c, res["best_bits"]))
        assert res["trace"][-1] == res["best_e"].min()


def test_anneal_zero_temperature_ends_in_local_minimum():
    c = _canon(_rand_int_instance(4, 20, 3))
    res = oracle.anneal(c, n_rep=64, sweeps=30, t_start=1e-9, t_end=1e-9, seed=5)
    _, de = oracle.fields(c, res["final_bits"])
    assert (de >= 0).all()


def test_anneal_given_init_and_determinism():
    c = _canon(_rand_int_instance(6, 18, 3))
    x0 = W.pack_bits(W.random_states(18, 32, seed=3))
    a = oracle.anneal(c, 32, 10, 3.0, 0.1, seed=9, init_bits=x0)
    b = oracle.anneal(c, 32, 10, 3.0, 0.1, seed=9, init_bits=x0)
    np.testing.assert_array_equal(a["final_bits"], b["final_bits"])
    np.testing.assert_array_equal(a["best_e"], b["best_e"])
    # zero sweeps: final = best = init
    z = oracle.anneal(c, 32, 0, 3.0, 0.1, seed=9, init_bits=x0)
    np.testing.assert_array_equal(z["final_bits"], x0)
    np.testing.assert_array_equal(z["best_e"], oracle.energy(c, x0))


def test_anneal_schedule_split_matches_whole_run():
    """Sweeps [0, 11) then [11, 25) of one 25-sweep schedule, the second part
    starting from the first part's final states, reach the whole run's final
    states; the better of the two parts' best energies is the whole run's."""
    terms = W.cfg_int3(seed=12, n=14)
    c = oracle.canonicalize(terms)
    whole = oracle.anneal(c, 40, 25, 3.0, 0.1, seed=4)
    a = oracle.anneal(c, 40, 11, 3.0, 0.1, seed=4, schedule_sweeps=25)
    b = oracle.anneal(c, 40, 14, 3.0, 0.1, seed=4, init_bits=a["final_bits"], first_sweep=11, schedule_sweeps=25)
    np.testing.assert_array_equal(b["final_bits"], whole["final_bits"])
    np.testing.assert_array_equal(np.minimum(a["best_e"], b["best_e"]), whole["best_e"])
    np.testing.assert_array_equal(np.minimum(a["trace"][-1], b["trace"]), whole["trace"][11:])
    with pytest.raises(ValueError):
        oracle.anneal(c, 4, 10, 3.0, 0.1, seed=4, first_sweep=20, schedule_sweeps=25)


# ------------------------------------------------ tolerance scales and schedule


def _hand_instance():
    """Four variables with hand-picked weights whose squares give whole sums:
    a_0 = 3, a_1 = -4, b_01 = 12, b_23 = 84, c_123 = 2."""
    p = W.RawPoly([((0,), 3.0), ((1,), -4.0), ((0, 1), 12.0), ((2, 3), 84.0), ((1, 2, 3), 2.0)])
    return _canon(W.poly_to_terms(4, p, False))


def test_active_scale_by_hand():
    """s(x) = (sum over monomials with every variable set of w_S^2)^(1/2),
    the floor of the relative-error criterion.  Hand values: x = 1100 keeps
    a_0, a_1, b_01 (9 + 16 + 144 = 13^2); x = 0011 keeps b_23 (84); x = 1111
    keeps all five (7229); x = 0 keeps none.  A sum of |w| (19 at 1100), a
    missing root (169) or an RMS over the active terms (13 / sqrt 3) all
    differ from these."""
    c = _hand_instance()
    x = np.array([[1, 1, 0, 0], [0, 0, 1, 1], [1, 1, 1, 1], [0, 0, 0, 0], [0, 1, 1, 1]], dtype=np.uint8)
    got = oracle.active_scale(c, W.pack_bits(x))
    want = [13.0, 84.0, math.sqrt(9 + 16 + 144 + 7056 + 4), 0.0, math.sqrt(16 + 7056 + 4)]
    np.testing.assert_allclose(got, want, rtol=1e-15, atol=0)


def test_field_scale_by_hand():
    """s_i(x) = (sum over monomials S containing i whose other variables are
    all set of w_S^2)^(1/2): the bit's own value does not enter.  At
    x = 0111: bit 0 sees a_0 and b_01 (9 + 144); bit 1 sees a_1 and c_123
    (16 + 4; b_01 is off since x_0 = 0); bits 2 and 3 see b_23 and c_123
    (7056 + 4).  At x = 0011 bit 0 sees a_0 only (3) even though x_0 = 0,
    and bit 1 sees a_1 and c_123 (20)."""
    c = _hand_instance()
    x = np.array([[0, 1, 1, 1], [0, 0, 1, 1], [0, 0, 0, 0]], dtype=np.uint8)
    got = oracle.field_scale(c, W.pack_bits(x))
    want = [[math.sqrt(153), math.sqrt(20), math.sqrt(7060), math.sqrt(7060)],
            [3.0, math.sqrt(20), 84.0, 84.0],
            [3.0, 4.0, 0.0, 0.0]]
    np.testing.assert_allclose(got, want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("t0,t1,S", [(5.0, 0.01, 1000), (2.0, 3.0, 7), (1.0, 1.0, 4), (0.5, 0.25, 2)])
def test_schedule_is_geometric_from_t_start_to_t_end(t0, t1, S):
    """The reading of Sec. II.D.1's cooling: S temperatures, the first t_start,
    the last t_end, every ratio T_{s+1}/T_s the same (t_end/t_start)^(1/(S-1))."""
    T = oracle.schedule(t0, t1, S)
    assert len(T) == S
    assert T[0] == t0
    assert abs(T[-1] - t1) <= 4e-16 * t1
    r = (t1 / t0) ** (1.0 / (S - 1))
    np.testing.assert_allclose(T[1:] / T[:-1], r, rtol=1e-13, atol=0)
    assert (np.diff(T) < 0).all() if t1 < t0 else (np.diff(T) >= 0).all()


def test_schedule_single_sweep_is_t_start():
    np.testing.assert_array_equal(oracle.schedule(3.0, 0.1, 1), [3.0])


def test_anneal_uses_the_schedule_temperature_each_sweep():
    """The chain runs at the schedule's temperature: one replica on one
    variable with a_0 = 1 starting at x = 0 flips up in sweep s iff
    u_s < exp(-1 / T_s), with u_s the acceptance draw of (replica 0, sweep s,
    bit 0) from Philox word 0 at counter (0, s, 0, 0), key (seed, 0)."""
    c = _canon(W.poly_to_terms(1, W.RawPoly([((0,), 1.0)]), False))
    S, seed = 6, 31
    T = oracle.schedule(4.0, 0.5, S)
    x = np.zeros((1, 1), dtype=np.uint64)
    for s in range(S):
        res = oracle.anneal(c, 1, 1, 4.0, 0.5, seed=seed, init_bits=x, first_sweep=s, schedule_sweeps=S)
        word = int(oracle.philox4x64(np.array([0, s, 0, 0], dtype=np.uint64), (seed, 0))[0])
        u = (word >> 11) * 2.0 ** -53
        up = int(x[0, 0]) == 0
        flips = (not up) or u < math.exp(-1.0 / T[s])  # dE = -1 going down is always taken
        assert int(res["final_bits"][0, 0]) == (int(x[0, 0]) ^ int(flips))
        x = res["final_bits"]


def _np_philox_word(ctr, key, lane):
    """Word `lane` of Philox4x64-10 at `ctr`, from numpy's generator (which
    increments its counter before the first block)."""
    words = [int(v) for v in ctr]
    for j in range(4):
        if words[j] > 0:
            words[j] -= 1
            break
        words[j] = 2 ** 64 - 1
    g = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(words, dtype=np.uint64))
    return int(g.random_raw(4)[lane])


def test_anneal_margins_by_hand():
    """The oracle's per-sweep decision margins, replayed in plain Python: the
    flip change from two energy sums (its definition), the acceptance draw
    from numpy's Philox, A = sum |w| over the active monomials containing the
    visited bit, margin = |dE beta + ln u| / (beta A) (Sec. II.D.1 acceptance
    u < exp(-dE beta)); the final states must agree as well."""
    rng = np.random.default_rng(5)
    n, B, S, seed = 6, 4, 3, 17
    monos = [m for r in (1, 2, 3) for m in itertools.combinations(range(n), r)]
    ws = [float(np.float32(v)) for v in rng.normal(size=len(monos))]
    terms = W.poly_to_terms(n, W.RawPoly(list(zip(monos, ws))), False)
    c = _canon(terms)
    x0 = rng.integers(0, 2, size=(B, n)).astype(np.uint8)
    res = oracle.anneal(c, B, S, 3.0, 0.3, seed=seed, init_bits=W.pack_bits(x0), margins=True)
    temps = oracle.schedule(3.0, 0.3, S)

    def energy(x):
        return math.fsum(w for m, w in zip(monos, ws) if all(x[v] for v in m))

    for b in range(B):
        x = [int(v) for v in x0[b]]
        for s in range(S):
            beta = 1.0 / temps[s]
            mm = math.inf
            for i in range(n):
                y = list(x)
                y[i] ^= 1
                de = energy(y) - energy(x)
                a = math.fsum(abs(w) for m, w in zip(monos, ws) if i in m and all(x[v] for v in m if v != i))
                u = (_np_philox_word((b, s, i // 4, 0), (seed, 0), i % 4) >> 11) * 2.0 ** -53
                if a > 0 and u > 0:
                    mm = min(mm, abs(de * beta + math.log(u)) / (beta * a))
                if de <= 0 or u < math.exp(-de * beta):
                    x = y
            assert res["margin"][b, s] == pytest.approx(mm, rel=1e-9, abs=1e-13)
        assert W.unpack_bits(res["final_bits"], n)[b].tolist() == x


# ---------------------------------------------------------- TT decomposition


def test_tt_svd_of_the_tsp_tensor(golden):
    """Sec. VI.F: the exact TT decomposition of the (6,)^6 TSP tensor has the
    printed core shapes (ranks 2, 3, 4, 4, 2), reproduces the tensor, gives
    every state's energy through the cores, and its contraction with the
    six x vectors has the printed einsum-path counts."""
    import oracle.tt as TT

    g = golden["tsp_intenc"]
    c = _canon(W.paper_tsp_intenc())
    h = oracle.paper_tensor(c).astype(np.float64)
    cores, ranks = TT.tt_svd(h)
    assert ranks == [2, 3, 4, 4, 2]
    shapes = [list(cores[0].shape[1:])] + [list(x.shape) for x in cores[1:-1]] + [list(cores[-1].shape[:2])]
    assert shapes == g["tt_core_shapes"]
    assert np.abs(TT.tt_full(cores) - h).max() < 1e-9
    x = W.all_states(6)
    np.testing.assert_allclose(TT.tt_energies(cores, x), oracle.energy(c, W.pack_bits(x)), rtol=0, atol=1e-9)
    v = np.ones(6)
    ops = [v] * 6 + [cores[0][0]] + [x for x in cores[1:-1]] + [cores[-1][:, :, 0]]
    _, text = np.einsum_path("i,j,k,l,m,n,iA,AjB,BkC,ClD,DmE,En->", *ops, optimize="greedy")
    t = g["einsum_tt"]
    assert f"{t['naive_flops']:.3e}" in text
    assert f"{t['optimized_flops']:.3e}" in text
    assert f"{t['largest_intermediate']:.3e}" in text


@pytest.mark.parametrize("seed,n,k,integer", [(1, 7, 3, True), (2, 5, 4, False), (3, 9, 2, True), (4, 4, 5, False)])
def test_tt_energies_equal_the_definition(seed, n, k, integer):
    """Random instances: the TT form's energies equal the term sums on every
    state (brute force), and each rank is the rank of its unfolding."""
    import oracle.tt as TT

    terms = _rand_int_instance(seed, n, k) if integer else _rand_real_instance(seed, n, k)
    c = _canon(terms)
    h = oracle.paper_tensor(c).astype(np.float64)
    cores, ranks = TT.tt_svd(h)
    d = h.ndim
    assert ranks == [int(np.linalg.matrix_rank(h.reshape(n ** j, -1))) for j in range(1, d)]
    x = W.all_states(n)
    want = oracle.energy(c, W.pack_bits(x))
    scale = np.abs(np.asarray(c.weights, dtype=np.float64)).sum()
    assert np.abs(TT.tt_energies(cores, x) - want).max() <= 1e-12 * scale * n ** 2


# ---------------------------------------------------------- gradient descent


@pytest.mark.parametrize("seed,n,k,integer", [(1, 6, 3, False), (2, 5, 4, True), (3, 8, 2, False)])
def test_gd_gradient_pins(seed, n, k, integer):
    """The oracle's gradient of the multilinear extension: equal to central
    finite differences (exact up to rounding, E being linear in each p_i);
    equal to the local field at binary points; the extension equals the
    energy at binary points."""
    import oracle.gd as G

    terms = _rand_int_instance(seed, n, k) if integer else _rand_real_instance(seed, n, k)
    c = _canon(terms)
    rng = np.random.default_rng(seed)
    p = rng.random((7, n))
    g = G.gradient(c, p)
    h = 1e-3
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        fd = (G.extension(c, p + e) - G.extension(c, p - e)) / (2 * h)
        np.testing.assert_allclose(g[:, i], fd, rtol=1e-9, atol=1e-9)
    x = W.random_states(n, 9, seed=seed)
    bits = W.pack_bits(x)
    np.testing.assert_allclose(G.gradient(c, x.astype(np.float64)), oracle.fields(c, bits)[0], rtol=0, atol=1e-12)
    np.testing.assert_allclose(G.extension(c, x.astype(np.float64)), oracle.energy(c, bits), rtol=0, atol=1e-12)


def test_gd_step_by_hand():
    """Two variables, E = 2 p0 - 3 p0 p1 + p1: g = (2 - 3 p1, 1 - 3 p0); one
    projected step from (0.5, 0.9) with eta 0.5 gives (0.5 - 0.5 (2 - 2.7),
    0.9 - 0.5 (1 - 1.5)) = (0.85, 1.15 -> 1.0); it rounds to (1, 1), E = 0."""
    import oracle.gd as G

    c = _canon(W.poly_to_terms(2, W.RawPoly([((0,), 2.0), ((0, 1), -3.0), ((1,), 1.0)]), False))
    p = G.descend(c, np.array([[0.5, 0.9]]), 1, 0.5)
    np.testing.assert_allclose(p, [[0.85, 1.0]], rtol=0, atol=1e-15)
    x, e = G.round_and_score(c, p)
    assert x.tolist() == [[1, 1]] and e.tolist() == [0.0]


def test_gd_random_start_uses_philox_tag_3():
    import oracle.gd as G

    p = G.random_start(6, 2, seed=11)
    for b in range(2):
        for i in range(6):
            word = _np_philox_word((b, 0, i // 4, 3), (11, 0), i % 4)
            assert p[b, i] == (word >> 11) * 2.0 ** -53
