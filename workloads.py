"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only *describes problems*: it writes cost polynomials as raw term
lists (index tuples with coefficients, repeated indices and duplicate
monomials allowed, constants allowed) and draws candidate bit vectors.  It
holds none of the solver's arithmetic: no canonicalisation (x*x = x, merging,
offset extraction), no energies, no fields, no search.  Both the CPU oracle
and the GPU library receive exactly the arrays produced here.

Problem families
----------------
* ``cfg_int3``  order-3, N=16, integer coefficients a_i, b_ij, c_ijk ~ U{-8..8}
  (all i<j<k present) -- the small bit-exact case.
* ``cfg_real3`` order-3, N=128, every a_i, b_ij (i<j), c_ijk (i<j<k) drawn
  ~N(0,1)/N and rounded to FP32 -- the dense real-valued case.
* ``cfg_intenc4`` integer-encoded order-4: 8 integers z_p in [0,63], each a
  6-bit binary code (bit index 6p+a, least significant first, the binary
  integer encoding y = sum_a 2^a x_a of the paper's Sec. IV.B); cost
  sum over 12 distinct pairs of w_pq (z_p z_q - t_pq)^2.
* ``cfg_mixed``  many instances with N ~ U{24..160}, order ~ U{2,3,4}; every
  sorted subset of size 1..k is present with probability 0.3 and carries an
  FP32 ~N(0,1) coefficient.
* The three worked problems of the paper's Sec. V (seating grid, Pythagorean
  triples, integer-encoded TSP constraint), written from their problem
  statements.

All randomness is numpy PCG64 (``numpy.random.default_rng``) from the given
seed, drawn in the documented order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# raw polynomials (problem statements, not canonical forms)
# --------------------------------------------------------------------------


class RawPoly:
    """A polynomial in binary variables kept as an *unsimplified* term list.

    Multiplication concatenates index tuples and multiplies coefficients;
    addition concatenates term lists.  Nothing is merged or reduced, so
    x_i * x_i stays a two-index term: reducing it is the solver's job.
    """

    __slots__ = ("terms",)

    def __init__(self, terms=None):
        self.terms = list(terms) if terms else []  # [(tuple(idx), coeff)]

    @staticmethod
    def var(i: int) -> "RawPoly":
        return RawPoly([((int(i),), 1)])

    @staticmethod
    def const(c) -> "RawPoly":
        return RawPoly([((), c)])

    def _coerce(self, o):
        return o if isinstance(o, RawPoly) else RawPoly.const(o)

    def __add__(self, o):
        o = self._coerce(o)
        return RawPoly(self.terms + o.terms)

    __radd__ = __add__

    def __neg__(self):
        return RawPoly([(t, -c) for t, c in self.terms])

    def __sub__(self, o):
        return self + (-self._coerce(o))

    def __rsub__(self, o):
        return self._coerce(o) + (-self)

    def __mul__(self, o):
        o = self._coerce(o)
        return RawPoly([(t1 + t2, c1 * c2) for t1, c1 in self.terms for t2, c2 in o.terms])

    __rmul__ = __mul__

    def __pow__(self, n: int):
        out = RawPoly.const(1)
        for _ in range(n):
            out = out * self
        return out


@dataclass
class TermList:
    """CSR term list: term t has indices term_idx[term_ptr[t]:term_ptr[t+1]]."""

    n_vars: int
    term_ptr: np.ndarray  # int64 [n_terms+1]
    term_idx: np.ndarray  # int32 [nnz]
    coeff: np.ndarray  # int64 or float64 [n_terms]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_terms(self) -> int:
        return len(self.coeff)

    @property
    def is_integer(self) -> bool:
        return self.coeff.dtype == np.int64

    def max_term_len(self) -> int:
        return int(np.max(np.diff(self.term_ptr))) if self.n_terms else 0


def poly_to_terms(n_vars: int, poly: RawPoly, integer: bool, name: str = "") -> TermList:
    ptr = [0]
    idx: list[int] = []
    co = []
    for t, c in poly.terms:
        idx.extend(t)
        ptr.append(len(idx))
        co.append(c)
    coeff = np.array(co, dtype=np.int64 if integer else np.float64)
    return TermList(n_vars, np.array(ptr, dtype=np.int64), np.array(idx, dtype=np.int32), coeff, name)


def subsets_to_terms(n_vars: int, subsets: list[np.ndarray], coeffs: list[np.ndarray],
                     integer: bool, name: str = "") -> TermList:
    """Term list from per-order arrays of index tuples ([M_r, r]) and coefficients."""
    ptr_parts = [np.zeros(1, dtype=np.int64)]
    idx_parts = []
    co_parts = []
    base = 0
    for s, c in zip(subsets, coeffs):
        m, r = s.shape
        if m == 0:
            continue
        ptr_parts.append(base + r * np.arange(1, m + 1, dtype=np.int64))
        base += r * m
        idx_parts.append(s.reshape(-1).astype(np.int32))
        co_parts.append(np.asarray(c))
    ptr = np.concatenate(ptr_parts)
    idx = np.concatenate(idx_parts) if idx_parts else np.zeros(0, np.int32)
    dt = np.int64 if integer else np.float64
    co = np.concatenate(co_parts).astype(dt) if co_parts else np.zeros(0, dt)
    return TermList(n_vars, ptr, idx, co, name)


# --------------------------------------------------------------------------
# combinations (lexicographic), vectorised
# --------------------------------------------------------------------------


def lex_subsets(n: int, r: int) -> np.ndarray:
    """All r-subsets of range(n) as sorted rows, lexicographic order, [C(n,r), r]."""
    if r == 0:
        return np.zeros((1, 0), dtype=np.int32)
    if r == 1:
        return np.arange(n, dtype=np.int32)[:, None]
    rows = []
    for first in range(n - r + 1):
        rest = lex_subsets(n - first - 1, r - 1) + (first + 1)
        rows.append(np.concatenate([np.full((len(rest), 1), first, np.int32), rest.astype(np.int32)], axis=1))
    return np.concatenate(rows, axis=0) if rows else np.zeros((0, r), np.int32)


def colex_unrank(ranks: np.ndarray, n: int, r: int) -> np.ndarray:
    """Sorted r-subsets of range(n) with the given colexicographic ranks."""
    ranks = np.asarray(ranks, dtype=np.int64).copy()
    out = np.zeros((len(ranks), r), dtype=np.int32)
    for j in range(r, 0, -1):
        table = np.array([math.comb(c, j) for c in range(n + 1)], dtype=np.int64)
        c = np.searchsorted(table, ranks, side="right") - 1
        out[:, j - 1] = c
        ranks -= table[c]
    return out


# --------------------------------------------------------------------------
# candidate bit vectors
# --------------------------------------------------------------------------


def random_states(n_vars: int, batch: int, seed: int) -> np.ndarray:
    """[batch, n_vars] uint8 iid Bernoulli(1/2) bits."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, size=(batch, n_vars), dtype=np.uint8)


def all_states(n_vars: int) -> np.ndarray:
    """[2^n, n] uint8; row b holds the binary digits of b (variable i = bit i)."""
    b = np.arange(1 << n_vars, dtype=np.int64)
    return ((b[:, None] >> np.arange(n_vars)[None, :]) & 1).astype(np.uint8)


def pack_bits(x: np.ndarray) -> np.ndarray:
    """[B, N] 0/1 -> [W, B] uint64 word-major; variable i in word i>>6 at bit i&63."""
    x = np.asarray(x, dtype=np.uint64)
    bsz, n = x.shape
    w = (n + 63) // 64
    out = np.zeros((w, bsz), dtype=np.uint64)
    for i in range(n):
        out[i >> 6] |= x[:, i] << np.uint64(i & 63)
    return out


def unpack_bits(words: np.ndarray, n_vars: int) -> np.ndarray:
    """Inverse of :func:`pack_bits`."""
    words = np.asarray(words, dtype=np.uint64)
    bsz = words.shape[1]
    out = np.zeros((bsz, n_vars), dtype=np.uint8)
    for i in range(n_vars):
        out[:, i] = ((words[i >> 6] >> np.uint64(i & 63)) & np.uint64(1)).astype(np.uint8)
    return out


# --------------------------------------------------------------------------
# benchmark-style instance families
# --------------------------------------------------------------------------


def cfg_int3(seed: int, n: int = 16) -> TermList:
    """Order 3, all a_i, b_ij (i<j), c_ijk (i<j<k) ~ U{-8..8} (int)."""
    rng = np.random.default_rng(seed)
    subs = [lex_subsets(n, r) for r in (1, 2, 3)]
    co = [rng.integers(-8, 9, size=len(s)).astype(np.int64) for s in subs]
    t = subsets_to_terms(n, subs, co, True, f"int3_n{n}_s{seed}")
    t.meta.update(order=3, family="int3")
    return t


def cfg_real3(seed: int, n: int = 128, cubic_only: bool = False) -> TermList:
    """Order 3, every sorted subset of size 1..3 (or only 3) with FP32 N(0,1)/n."""
    rng = np.random.default_rng(seed)
    orders = (3,) if cubic_only else (1, 2, 3)
    subs = [lex_subsets(n, r) for r in orders]
    co = [(rng.standard_normal(len(s)) / n).astype(np.float32).astype(np.float64) for s in subs]
    t = subsets_to_terms(n, subs, co, False, f"real3_n{n}_s{seed}")
    t.meta.update(order=3, family="real3")
    return t


def cfg_intenc4(seed: int, n_int: int = 8, bits: int = 6, n_pairs: int = 12) -> TermList:
    """Sum over distinct pairs of w (z_p z_q - t)^2 with z_p = sum_a 2^a x_{bits*p+a}."""
    rng = np.random.default_rng(seed)
    all_pairs = [(p, q) for p in range(n_int) for q in range(p + 1, n_int)]
    pick = rng.choice(len(all_pairs), size=n_pairs, replace=False)
    w = rng.integers(1, 5, size=n_pairs)
    zmax = (1 << bits) - 1
    t = rng.integers(0, zmax * zmax + 1, size=n_pairs)
    z = [sum((RawPoly.var(bits * p + a) * (1 << a) for a in range(bits)), RawPoly()) for p in range(n_int)]
    h = RawPoly()
    for m, pi in enumerate(pick):
        p, q = all_pairs[pi]
        h = h + int(w[m]) * (z[p] * z[q] - int(t[m])) ** 2
    tl = poly_to_terms(n_int * bits, h, True, f"intenc4_s{seed}")
    tl.meta.update(order=4, family="intenc4", pairs=[all_pairs[i] for i in pick], w=w.tolist(), t=t.tolist())
    return tl


def cfg_mixed_instance(master_seed: int, index: int, n_lo: int = 24, n_hi: int = 160,
                       orders=(2, 3, 4), density: float = 0.3) -> TermList:
    """Instance ``index`` of the mixed family (independent stream per index)."""
    rng = np.random.default_rng([master_seed, index])
    n = int(rng.integers(n_lo, n_hi + 1))
    k = int(rng.choice(orders))
    subs, co = [], []
    for r in range(1, k + 1):
        total = math.comb(n, r)
        keep = np.nonzero(rng.random(total) < density)[0]
        subs.append(colex_unrank(keep, n, r))
        co.append(rng.standard_normal(len(keep)).astype(np.float32).astype(np.float64))
    t = subsets_to_terms(n, subs, co, False, f"mixed_{master_seed}_{index}")
    t.meta.update(order=k, family="mixed")
    return t


# --------------------------------------------------------------------------
# the paper's worked problems (Sec. V), written from their statements
# --------------------------------------------------------------------------


def pseudo_boolean_terms(n_vars: int, values: np.ndarray, name: str = "") -> TermList:
    """The unique multilinear polynomial that takes values[m] at the state
    whose bit i is bit i of m (all 2^n states, integers): its coefficients
    are the Moebius transform of the values over the subset lattice,
    w_S = sum over T subset of S of (-1)^(|S|-|T|) f(T); the empty set's
    coefficient is the offset."""
    w = np.array(values, dtype=np.int64).copy()
    if w.shape != (1 << n_vars,):
        raise ValueError("one value per state")
    for i in range(n_vars):
        bit = 1 << i
        idx = np.nonzero(np.arange(1 << n_vars) & bit)[0]
        w[idx] -= w[idx ^ bit]
    masks = np.nonzero(w)[0]
    subsets = {}
    for m in masks:
        vs = [i for i in range(n_vars) if (int(m) >> i) & 1]
        subsets.setdefault(len(vs), []).append((vs, int(w[m])))
    subs, co = [], []
    for r in sorted(subsets):
        rows = [v for v, _ in subsets[r]]
        subs.append(np.zeros((len(rows), 0), dtype=np.int64) if r == 0 else np.array(rows, dtype=np.int64))
        co.append(np.array([c for _, c in subsets[r]], dtype=np.int64))
    return subsets_to_terms(n_vars, subs, co, True, name=name)


def paper_seating(grid: int = 5, run: int = 3, penalty: int = 10) -> TermList:
    """Sec. V.A: `grid` x `grid` seats; one point for every occupied seat and
    a penalty for every `run` consecutive occupied seats along a row or a
    column: cost = -(occupied seats) + penalty x (fully occupied windows).
    Variable of seat (i, j) is i*grid + j."""
    windows = [[i * grid + j + d for d in range(run)] for i in range(grid) for j in range(grid - run + 1)]
    windows += [[(i + d) * grid + j for d in range(run)] for j in range(grid) for i in range(grid - run + 1)]
    singles = np.arange(grid * grid, dtype=np.int64).reshape(-1, 1)
    t = subsets_to_terms(grid * grid, [singles, np.array(windows, dtype=np.int64)],
                         [-np.ones(grid * grid, dtype=np.int64), np.full(len(windows), penalty, dtype=np.int64)],
                         True, name="paper_seating")
    t.meta.update(order=run, family="paper")
    return t


def paper_pythagorean(bits: int = 4, penalty: int = 10) -> TermList:
    """Sec. V.B: integers x, y, z, each a `bits`-bit binary code (Sec. IV.B:
    bit a of integer p is variable p*bits + a, weight 2^a); the cost is
    (x^2 + y^2 - z^2)^2 plus `penalty` for each integer that is 0.  The terms
    are the multilinear expansion of that cost over all 2^(3 bits) states."""
    n = 3 * bits
    m = np.arange(1 << n, dtype=np.int64)
    ints = [(m >> (p * bits)) & ((1 << bits) - 1) for p in range(3)]
    f = (ints[0] ** 2 + ints[1] ** 2 - ints[2] ** 2) ** 2 + penalty * sum((v == 0).astype(np.int64) for v in ints)
    t = pseudo_boolean_terms(n, f, "paper_pythagorean")
    t.meta.update(order=4, family="paper", bits=bits)
    return t


def paper_tsp_intenc(penalty: int = 10, target: int = 6) -> TermList:
    """Sec. V.C: three 2-bit integers x_p = 2 q_{p,0} + q_{p,1} (the first
    bit is the more significant one); cost penalty * (x_B x_C x_D - target)^2.
    The formulation declares a fourth, unused integer; only the six used bits
    are variables here (variable 2p + a for q_{p,a}), which is the paper's
    dimension reduction of Sec. IV.D.  The terms are the multilinear expansion
    of the cost over all 64 states."""
    m = np.arange(64, dtype=np.int64)
    xs = [2 * ((m >> (2 * p)) & 1) + ((m >> (2 * p + 1)) & 1) for p in range(3)]
    f = penalty * (xs[0] * xs[1] * xs[2] - target) ** 2
    t = pseudo_boolean_terms(6, f, "paper_tsp")
    t.meta.update(order=6, family="paper")
    return t


def decode_int(bits_row: np.ndarray, first_var: int, n_bits: int, msb_first: bool = False) -> int:
    """Value of an integer encoded by variables first_var .. first_var+n_bits-1."""
    v = 0
    for a in range(n_bits):
        b = int(bits_row[first_var + a])
        v += b << ((n_bits - 1 - a) if msb_first else a)
    return v


# --------------------------------------------------------------------------
# flip-proposal network: initial weights
# --------------------------------------------------------------------------

MLP_HIDDEN = 256
MLP_FEATURES = 3
MLP_PARAMS = MLP_FEATURES * MLP_HIDDEN + 2 * MLP_HIDDEN + 1


def mlp_init(seed: int) -> np.ndarray:
    """FP32 parameter vector of the 3 -> 256 -> 1 proposal network, Glorot
    uniform matrices and zero biases: W1[f][u] at f*256+u, b1 at 768, W2 at
    1024, b2 at 1280."""
    rng = np.random.default_rng(seed)
    a1 = np.sqrt(6.0 / (MLP_FEATURES + MLP_HIDDEN))
    a2 = np.sqrt(6.0 / (MLP_HIDDEN + 1))
    p = np.zeros(MLP_PARAMS, dtype=np.float32)
    p[:MLP_FEATURES * MLP_HIDDEN] = rng.uniform(-a1, a1, MLP_FEATURES * MLP_HIDDEN)
    p[MLP_FEATURES * MLP_HIDDEN + MLP_HIDDEN:MLP_FEATURES * MLP_HIDDEN + 2 * MLP_HIDDEN] = rng.uniform(-a2, a2,
                                                                                                     MLP_HIDDEN)
    return p


def mlp_samples(m: int, seed: int, p_pos: float = 0.3) -> tuple[np.ndarray, np.ndarray]:
    """Synthetic (features [m][3] FP32, labels [m] FP32) with the value ranges
    of recorded transitions: x in {0,1}, beta*dE ~ N(0, 3^2), beta*||H|| in
    [0.1, 20]; labels Bernoulli(p_pos)."""
    rng = np.random.default_rng(seed)
    f = np.zeros((m, MLP_FEATURES), dtype=np.float32)
    f[:, 0] = rng.integers(0, 2, m)
    f[:, 1] = rng.normal(0.0, 3.0, m)
    f[:, 2] = rng.uniform(0.1, 20.0, m)
    y = (rng.random(m) < p_pos).astype(np.float32)
    return f, y
