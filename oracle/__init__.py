"""CPU oracle for the HOBO hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct implementations of what the GPU library
computes, written from the paper (arXiv 2407.19987, "HOBOTAN"):

* :func:`canonicalize`   -- a raw term list to canonical monomials + offset
  (Sec. II.B polynomial; Sec. III.C / IV.A say every term is a coefficient
  on a product of binary variables, x*x = x for binary x).
* :func:`energy`         -- E(x) = sum_S w_S prod_{i in S} x_i per row of a
  batch (Sec. II.C contraction; Sec. IV.C batch of vectors).  Exact: integer
  instances in int64, real ones summed exactly and rounded once to FP64.
* :func:`fields`         -- local fields g_i and single-flip changes
  dE_i = E(x xor e_i) - E(x) = (1 - 2 x_i) g_i.
* :func:`paper_tensor`   -- the dense order-k HOBO tensor in the paper's
  layout: a term of lower order is stored at the index tuple that repeats its
  smallest variable until the tuple has k entries (Sec. III.C, IV.A).
* :func:`qubo_matrix`    -- the upper-triangular Q of an order-2 instance
  (Sec. II.B QUBO form), E = x^T Q x.
* :func:`brute_force`    -- exhaustive minimum over all 2^N states.
* :func:`anneal`         -- batched single-flip Metropolis annealing
  (Sec. II.D.1) with the readings documented in oracle.c.
* :func:`philox4x64`     -- Philox4x64-10 counter-based generator.
* :mod:`oracle.mlp`      -- FP64 forward/backward of the flip-proposal MLP.

Nothing here imports, links or calls the GPU library, and the GPU library
never imports this package.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP over replicas)."""
    import subprocess

    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        subprocess.run(
            ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC", src, "-o", _LIB_PATH, "-lm"],
            check=True,
        )
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint64
        lib.orc_energy.argtypes = [i32, i32, P, P, P, i32, i64, P, P, P]
        lib.orc_energy.restype = i32
        lib.orc_fields.argtypes = [i32, i32, P, P, P, i32, i64, P, P, P, P, P]
        lib.orc_fields.restype = i32
        lib.orc_brute_force.argtypes = [i32, i32, P, P, P, P, P, P, P, i64]
        lib.orc_brute_force.restype = i32
        lib.orc_philox4x64.argtypes = [P, P, P]
        lib.orc_philox4x64.restype = None
        lib.orc_anneal.argtypes = [i32, i32, P, P, P, i32, i64, i32, P, u64, u64, i32, P, P, P, P, P, P, P, i32, P]
        lib.orc_anneal.restype = i32
        lib.orc_num_threads.argtypes = []
        lib.orc_num_threads.restype = i32
        lib.orc_set_threads.argtypes = [i32]
        lib.orc_set_threads.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's later parallel loops (for timing)."""
    _load().orc_set_threads(int(n))


# --------------------------------------------------------------------------
# canonical form
# --------------------------------------------------------------------------


@dataclass
class Canonical:
    """Canonical instance: distinct sorted monomials with non-zero weights."""

    n_vars: int
    order: int
    monos: list  # list[tuple[int, ...]], each sorted, distinct, non-empty
    weights: list  # python int or float per monomial
    offset: object  # python int or float
    integer: bool

    # fixed-point view used by the C routines
    def csr(self):
        ptr = np.zeros(len(self.monos) + 1, dtype=np.int64)
        for m, s in enumerate(self.monos):
            ptr[m + 1] = ptr[m] + len(s)
        idx = np.array([i for s in self.monos for i in s], dtype=np.int32)
        return ptr, idx

    def fixed(self):
        """(int64 coefficients, scale s) with weight = coeff * 2^-s exactly."""
        if self.integer:
            return np.array(self.weights, dtype=np.int64), 0
        s = 0
        for w in self.weights:
            m, e = math.frexp(w)  # w = m * 2^e, 0.5 <= |m| < 1
            mi = int(m * (1 << 53))
            tz = (mi & -mi).bit_length() - 1 if mi else 0
            s = max(s, 53 - e - tz)
        ints = [int(w * (2.0 ** s)) if abs(w * 2.0 ** s) < 2 ** 53 else _exact_scale(w, s) for w in self.weights]
        big = max((abs(v) for v in ints), default=0)
        if big >= 2 ** 62 or big * max(len(ints), 1) >= 2 ** 125:
            raise ValueError("oracle: coefficient dynamic range too wide for exact fixed point")
        return np.array(ints, dtype=np.int64), s


def _exact_scale(w: float, s: int) -> int:
    m, e = math.frexp(w)
    mi = int(m * (1 << 53))
    sh = e - 53 + s
    return mi << sh if sh >= 0 else mi >> (-sh)


def canonicalize(terms) -> Canonical:
    """Raw term list -> canonical monomials (Sec. II.B / III.C).

    Each term's index multiset becomes a set (x_i^2 = x_i for binary x);
    terms with the same set are summed; the empty set goes to the offset;
    zero sums are dropped.  The order k is the largest monomial size.
    """
    integer = terms.coeff.dtype == np.int64
    acc: dict = {}
    offset_parts = []
    ptr, idx, co = terms.term_ptr, terms.term_idx, terms.coeff
    for t in range(len(co)):
        key = tuple(sorted(set(int(v) for v in idx[ptr[t]:ptr[t + 1]])))
        c = int(co[t]) if integer else float(co[t])
        if len(key) == 0:
            offset_parts.append(c)
        else:
            acc.setdefault(key, []).append(c)
    monos, weights = [], []
    for key in sorted(acc.keys(), key=lambda k: (len(k), k)):
        w = sum(acc[key]) if integer else math.fsum(acc[key])
        if w != 0:
            if integer and not (-(2 ** 63) <= w < 2 ** 63):
                raise OverflowError("oracle: integer coefficient outside int64")
            monos.append(key)
            weights.append(w)
    offset = sum(offset_parts) if integer else math.fsum(offset_parts)
    order = max((len(m) for m in monos), default=0)
    return Canonical(terms.n_vars, order, monos, weights, offset, integer)


# --------------------------------------------------------------------------
# energies and fields
# --------------------------------------------------------------------------


def _bits_arg(canon: Canonical, bits: np.ndarray):
    bits = np.ascontiguousarray(bits, dtype=np.uint64)
    assert bits.ndim == 2 and bits.shape[0] == (canon.n_vars + 63) // 64
    return bits, bits.shape[1]


def energy(canon: Canonical, bits: np.ndarray):
    """Energies (offset excluded) of the rows of a [W][B] bit matrix.

    int64 array for integer instances, correctly rounded float64 otherwise.
    """
    bits, B = _bits_arg(canon, bits)
    ptr, idx = canon.csr()
    co, s = canon.fixed()
    lib = _load()
    if canon.integer:
        out = np.zeros(B, dtype=np.int64)
        rc = lib.orc_energy(canon.n_vars, len(co), _p(ptr), _p(idx), _p(co), s, B, _p(bits), _p(out), None)
        if rc != 0:
            raise OverflowError("oracle: energy outside int64")
        return out
    out = np.zeros(B, dtype=np.float64)
    lib.orc_energy(canon.n_vars, len(co), _p(ptr), _p(idx), _p(co), s, B, _p(bits), None, _p(out))
    return out


def fields(canon: Canonical, bits: np.ndarray):
    """(g, dE), each [B][N]: local fields and single-flip energy changes."""
    bits, B = _bits_arg(canon, bits)
    ptr, idx = canon.csr()
    co, s = canon.fixed()
    n = canon.n_vars
    lib = _load()
    if canon.integer:
        g = np.zeros((B, n), dtype=np.int64)
        de = np.zeros((B, n), dtype=np.int64)
        rc = lib.orc_fields(n, len(co), _p(ptr), _p(idx), _p(co), s, B, _p(bits), _p(g), None, _p(de), None)
        if rc != 0:
            raise OverflowError("oracle: field outside int64")
        return g, de
    g = np.zeros((B, n), dtype=np.float64)
    de = np.zeros((B, n), dtype=np.float64)
    lib.orc_fields(n, len(co), _p(ptr), _p(idx), _p(co), s, B, _p(bits), None, _p(g), None, _p(de))
    return g, de


def _rows(canon: Canonical, bits: np.ndarray) -> np.ndarray:
    bits = np.asarray(bits, dtype=np.uint64)
    n = canon.n_vars
    x = np.zeros((bits.shape[1], n), dtype=bool)
    for i in range(n):
        x[:, i] = ((bits[i >> 6] >> np.uint64(i & 63)) & np.uint64(1)).astype(bool)
    return x


def active_scale(canon: Canonical, bits: np.ndarray) -> np.ndarray:
    """s(x) = sqrt(sum over active monomials of w_S^2): the size of the terms
    that make up E(x), used as the floor of the relative error criterion
    (a tolerance scale, summed in plain double precision)."""
    x = _rows(canon, bits)
    out = np.zeros(x.shape[0])
    by_len: dict = {}
    for m, w in zip(canon.monos, canon.weights):
        by_len.setdefault(len(m), ([], []))
        by_len[len(m)][0].append(m)
        by_len[len(m)][1].append(float(w) ** 2)
    for r, (ms, w2) in by_len.items():
        idx = np.array(ms, dtype=np.int64)
        w2 = np.array(w2)
        for b0 in range(0, x.shape[0], 256):
            xb = x[b0:b0 + 256]
            act = np.ones((xb.shape[0], len(ms)), dtype=bool)
            for q in range(r):
                act &= xb[:, idx[:, q]]
            out[b0:b0 + 256] += act.astype(np.float64) @ w2
    return np.sqrt(out)


def field_scale(canon: Canonical, bits: np.ndarray) -> np.ndarray:
    """[B][N] sqrt(sum over monomials S containing i with S minus i active of
    w_S^2): the tolerance scale of the field g_i (plain double precision)."""
    x = _rows(canon, bits)
    n = canon.n_vars
    out = np.zeros((x.shape[0], n))
    by_len: dict = {}
    for m, w in zip(canon.monos, canon.weights):
        by_len.setdefault(len(m), ([], []))
        by_len[len(m)][0].append(m)
        by_len[len(m)][1].append(float(w) ** 2)
    for r, (ms, w2) in by_len.items():
        idx = np.array(ms, dtype=np.int64)
        w2 = np.array(w2)
        for p in range(r):
            onehot = np.zeros((len(ms), n))
            onehot[np.arange(len(ms)), idx[:, p]] = 1.0
            weighted = onehot * w2[:, None]
            for b0 in range(0, x.shape[0], 256):
                xb = x[b0:b0 + 256]
                act = np.ones((xb.shape[0], len(ms)), dtype=bool)
                for q in range(r):
                    if q != p:
                        act &= xb[:, idx[:, q]]
                out[b0:b0 + 256] += act.astype(np.float64) @ weighted
    return np.sqrt(out)


# --------------------------------------------------------------------------
# the paper's dense tensor layout and the QUBO matrix
# --------------------------------------------------------------------------


def paper_index(mono: tuple, k: int) -> tuple:
    """Index tuple of a monomial in the order-k tensor: the smallest variable
    is repeated at the front until the tuple has k entries (Sec. III.C, e.g.
    c_ijk -> c_iiijk at order 5)."""
    return (mono[0],) * (k - len(mono)) + tuple(mono)


def paper_tensor(canon: Canonical, k: int | None = None) -> np.ndarray:
    """Dense N^k HOBO tensor in the paper's layout (small N only)."""
    k = canon.order if k is None else k
    n = canon.n_vars
    if n ** k > (1 << 26):
        raise ValueError("paper_tensor: N^k too large")
    h = np.zeros((n,) * k, dtype=np.int64 if canon.integer else np.float64)
    for mono, w in zip(canon.monos, canon.weights):
        h[paper_index(mono, k)] = w
    return h


def tensor_contract(h: np.ndarray, x_rows: np.ndarray) -> np.ndarray:
    """E_b = sum_{i,j,k,...} H_{ijk...} x_{b,i} x_{b,j} x_{b,k} ... (Sec. IV.C)
    contracted one index at a time (each step is a library matmul)."""
    x = np.asarray(x_rows, dtype=np.float64)
    out = []
    for row in x:
        t = h.astype(np.float64)
        while t.ndim > 0:
            t = t @ row  # contracts the last index
        out.append(float(t))
    return np.array(out)


def qubo_matrix(canon: Canonical) -> np.ndarray:
    """Upper-triangular Q with Q_ii = a_i, Q_ij = b_ij (i < j): E = x^T Q x
    for binary x (Sec. II.B QUBO form)."""
    if canon.order > 2:
        raise ValueError("qubo_matrix: order > 2")
    n = canon.n_vars
    q = np.zeros((n, n), dtype=np.int64 if canon.integer else np.float64)
    for mono, w in zip(canon.monos, canon.weights):
        if len(mono) == 1:
            q[mono[0], mono[0]] += w
        else:
            q[mono[0], mono[1]] += w
    return q


# --------------------------------------------------------------------------
# exhaustive search
# --------------------------------------------------------------------------


def brute_force(canon: Canonical, cap: int = 64):
    """(min energy, number of minimisers, [minimiser as int]) over all 2^N."""
    ptr, idx = canon.csr()
    co, s = canon.fixed()
    mh = np.zeros(1, dtype=np.int64)
    ml = np.zeros(1, dtype=np.uint64)
    nm = np.zeros(1, dtype=np.int64)
    arg = np.zeros(cap, dtype=np.uint64)
    rc = _load().orc_brute_force(canon.n_vars, len(co), _p(ptr), _p(idx), _p(co), _p(mh), _p(ml), _p(nm), _p(arg), cap)
    if rc != 0:
        raise ValueError("brute_force: too many variables")
    v = (int(mh[0]) << 64) | int(ml[0])
    best = v if canon.integer else math.ldexp(float(v), -s)
    return best, int(nm[0]), [int(a) for a in arg[: min(cap, int(nm[0]))]]


# --------------------------------------------------------------------------
# RNG and annealing
# --------------------------------------------------------------------------


def philox4x64(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    o = np.zeros(4, dtype=np.uint64)
    _load().orc_philox4x64(_p(c), _p(k), _p(o))
    return o


def schedule(t_start: float, t_end: float, sweeps: int) -> np.ndarray:
    """Geometric temperatures T_s = T0 (T1/T0)^(s/(S-1)), s = 0..S-1."""
    if sweeps == 1:
        return np.array([t_start], dtype=np.float64)
    return np.array([t_start * (t_end / t_start) ** (s / (sweeps - 1)) for s in range(sweeps)], dtype=np.float64)


def anneal(canon: Canonical, n_rep: int, sweeps: int, t_start: float, t_end: float, seed: int,
           inst: int = 0, init_bits: np.ndarray | None = None, attempt: np.ndarray | None = None,
           first_sweep: int = 0, schedule_sweeps: int = 0, margins: bool = False):
    """Batched Metropolis annealing; see orc_anneal in oracle.c for the rules.

    Runs sweeps first_sweep .. first_sweep+sweeps-1 of a geometric schedule of
    schedule_sweeps sweeps (default: the whole schedule, first_sweep 0); the
    sweep index is the one of the schedule (temperature and random draws).
    Returns dict(final_bits [W][B], best_bits [W][B], best_e (exact, int64 or
    float64), trace [S], accepts); the best state starts at the start state.
    With margins=True also margin [B][S]: per replica and sweep the smallest
    relative decision margin |dE beta + ln u| / (beta A) (A = sum of |w| of
    the active monomials of the visited bit), the fraction of A by which an
    inexact dE may err before it could change a decision of that sweep."""
    n = canon.n_vars
    w = (n + 63) // 64
    ptr, idx = canon.csr()
    co, s = canon.fixed()
    total = schedule_sweeps if schedule_sweeps else sweeps
    if first_sweep + sweeps > total:
        raise ValueError("anneal: sweeps run past the schedule")
    temps = np.ascontiguousarray(schedule(t_start, t_end, total)[first_sweep:first_sweep + sweeps])
    bits = np.zeros((w, n_rep), dtype=np.uint64) if init_bits is None else np.array(init_bits, dtype=np.uint64)
    best_bits = np.zeros((w, n_rep), dtype=np.uint64)
    bh = np.zeros(n_rep, dtype=np.int64)
    bl = np.zeros(n_rep, dtype=np.uint64)
    trace = np.zeros(max(sweeps, 1), dtype=np.float64)
    nacc = np.zeros(1, dtype=np.int64)
    att = None if attempt is None else np.ascontiguousarray(attempt, dtype=np.uint8)
    marg = np.full((n_rep, max(sweeps, 1)), np.inf, dtype=np.float64) if margins else None
    rc = _load().orc_anneal(n, len(co), _p(ptr), _p(idx), _p(co), s, n_rep, sweeps, _p(temps), seed, inst,
                            1 if init_bits is not None else 0, _p(bits), _p(best_bits), _p(bh), _p(bl),
                            _p(trace), None if att is None else _p(att), _p(nacc), int(first_sweep),
                            None if marg is None else _p(marg))
    if rc != 0:
        raise ValueError("anneal: bad arguments")
    vals = [(int(h) << 64) | int(l) for h, l in zip(bh, bl)]
    vals = [v - (1 << 128) if v >= (1 << 127) else v for v in vals]
    best = np.array(vals, dtype=np.int64) if canon.integer else np.array([math.ldexp(float(v), -s) for v in vals])
    out = dict(final_bits=bits, best_bits=best_bits, best_e=best, trace=trace[:sweeps], accepts=int(nacc[0]))
    if margins:
        out["margin"] = marg[:, :sweeps]
    return out


# --------------------------------------------------------------------------
# result list of a sampling run
# --------------------------------------------------------------------------


def aggregate(n_vars: int, bits: np.ndarray, energies) -> list:
    """The paper's result list (Sec. V result blocks): every distinct sampled
    state with its energy and number of occurrences, ordered by energy, then
    by the bit sequence (x_0, x_1, ...).  bits [W][B]; returns a list of
    (bit tuple, energy, count, first sample index)."""
    w = np.asarray(bits, dtype=np.uint64)
    B = w.shape[1]
    rows = {}
    for b in range(B):
        key = tuple((int(w[i >> 6, b]) >> (i & 63)) & 1 for i in range(n_vars))
        e = energies[b]
        if key in rows:
            if rows[key][0] != e:
                raise ValueError("one state with two energies")
            rows[key][1] += 1
        else:
            rows[key] = [e, 1, b]
    return sorted(((k, v[0], v[1], v[2]) for k, v in rows.items()), key=lambda r: (r[1], r[0]))
