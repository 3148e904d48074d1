"""Symbolic front-end of the HOBO engine: binary symbols, polynomial
expressions over them, integer encodings, the compile step that turns an
expression into a tensor handle, and the sampling step that returns the
paper's result list.

* Expressions (Sec. II.B, III.C): a `Poly` is a sum of coefficient x product
  of binary symbols, kept with x*x = x applied, so that +, -, * and integer
  powers of expressions stay multilinear; numpy object arrays of symbols work
  with np.prod / np.sum.
* Integer encoding (Sec. IV.B): `int_var(n_bits)` is sum_k 2^k x_k over fresh
  symbols, k = 0 .. n_bits - 1 (least significant bit first).
* Compile (Sec. III.C / IV.A compile step, Sec. IV.D dimension reduction):
  `compile_hobo(expr)` keeps only the symbols the expression uses, numbers
  them 0 .. N-1 in declaration order, and builds the tensor through
  hobo_build_tensor; it returns the handle, the constant offset and the
  variable names.
* Sampling and results (Sec. V result blocks): `sample(compiled, shots)`
  anneals `shots` replicas on the GPU (hobo_anneal_batch), rescored exactly,
  and aggregates them (hobo_aggregate) into (state, energy, occurrences)
  rows, best first; a row decodes back to symbol values, arrays of symbols
  and encoded integers.

The arithmetic of the path (canonical form, device layouts, energies,
annealing) runs in the library; this module only expands expressions and
marshals term lists.
"""
from __future__ import annotations

import itertools
import numbers
import re
from dataclasses import dataclass, field

import numpy as np

from . import hobo

# symbol id -> name; ids grow in declaration order
_NAMES: list[str] = []


def _new_symbol(name: str) -> "Poly":
    _NAMES.append(name)
    return Poly({(len(_NAMES) - 1,): 1})


def symbol(name: str) -> "Poly":
    """One fresh binary symbol."""
    return _new_symbol(name)


def symbols_list(shape, fmt: str = "q{}") -> np.ndarray:
    """An array of fresh binary symbols of the given shape; the symbol at
    index (i, j, ...) is named fmt.format(i, j, ...)."""
    shape = (shape,) if isinstance(shape, numbers.Integral) else tuple(shape)
    out = np.empty(shape, dtype=object)
    for idx in itertools.product(*(range(s) for s in shape)):
        out[idx] = _new_symbol(fmt.format(*idx))
    return out


def int_var(n_bits: int, fmt: str = "z{}") -> "Poly":
    """Integer encoding (Sec. IV.B): y = sum_{k < n_bits} 2^k x_k over
    n_bits fresh symbols named fmt.format(k)."""
    if n_bits < 1:
        raise ValueError("n_bits must be >= 1")
    y = Poly()
    for k in range(n_bits):
        y = y + (1 << k) * _new_symbol(fmt.format(k))
    return y


def _num(c):
    if isinstance(c, (bool, np.bool_)):
        return int(c)
    if isinstance(c, numbers.Integral):
        return int(c)
    if isinstance(c, numbers.Real):
        return float(c)
    raise TypeError(f"coefficient {c!r} is not a real number")


class Poly:
    """Multilinear polynomial over binary symbols: {sorted symbol ids: coefficient}.
    The empty tuple holds the constant."""

    __slots__ = ("t",)
    __array_priority__ = 1000

    def __init__(self, terms=None):
        self.t = {}
        if terms:
            for k, v in terms.items():
                v = _num(v)
                if v != 0:
                    self.t[tuple(k)] = v

    @staticmethod
    def _lift(o) -> "Poly":
        if isinstance(o, Poly):
            return o
        return Poly({(): _num(o)})

    def __add__(self, o):
        if isinstance(o, np.ndarray):
            return NotImplemented
        o = Poly._lift(o)
        r = dict(self.t)
        for k, v in o.t.items():
            s = r.get(k, 0) + v
            if s == 0:
                r.pop(k, None)
            else:
                r[k] = s
        p = Poly()
        p.t = r
        return p

    __radd__ = __add__

    def __neg__(self):
        p = Poly()
        p.t = {k: -v for k, v in self.t.items()}
        return p

    def __sub__(self, o):
        if isinstance(o, np.ndarray):
            return NotImplemented
        return self + (-Poly._lift(o))

    def __rsub__(self, o):
        return Poly._lift(o) + (-self)

    def __mul__(self, o):
        if isinstance(o, np.ndarray):
            return NotImplemented
        o = Poly._lift(o)
        r = {}
        for ka, va in self.t.items():
            for kb, vb in o.t.items():
                k = tuple(sorted(set(ka) | set(kb)))  # x * x = x
                s = r.get(k, 0) + va * vb
                if s == 0:
                    r.pop(k, None)
                else:
                    r[k] = s
        p = Poly()
        p.t = r
        return p

    __rmul__ = __mul__

    def __pow__(self, n):
        if not isinstance(n, numbers.Integral) or n < 0:
            raise ValueError("only non-negative integer powers")
        out, base = Poly({(): 1}), self
        while n:
            if n & 1:
                out = out * base
            n >>= 1
            if n:
                base = base * base
        return out

    def __repr__(self):
        parts = []
        for k, v in sorted(self.t.items(), key=lambda kv: (len(kv[0]), kv[0])):
            parts.append(f"{v}" + "".join(f"*{_NAMES[i]}" for i in k))
        return " + ".join(parts) if parts else "0"

    @property
    def constant(self):
        return self.t.get((), 0)

    @property
    def order(self) -> int:
        return max((len(k) for k in self.t), default=0)

    def symbols(self) -> list[int]:
        return sorted({i for k in self.t for i in k})

    def value(self, assignment) -> float | int:
        """Value at an assignment {symbol id or name: 0/1} (symbols absent
        from it count as 0), or at a `Sample`."""
        if isinstance(assignment, Sample):
            assignment = assignment.by_id()
        named = {k: v for k, v in assignment.items() if isinstance(k, str)}
        def bit(i):
            if i in assignment:
                return int(assignment[i])
            return int(named.get(_NAMES[i], 0))
        return sum(v for k, v in self.t.items() if all(bit(i) for i in k))


@dataclass
class Compiled:
    """A compiled expression: the tensor handle (variables 0 .. N-1), its
    constant offset, and for each variable the symbol id and name."""
    tensor: "hobo.Tensor"
    offset: object
    symbol_ids: list
    names: list

    @property
    def n_vars(self) -> int:
        return len(self.symbol_ids)


def compile_hobo(expr, max_order: int = 0) -> Compiled:
    """Compile an expression into a tensor handle (hobo_build_tensor) with
    the unused symbols dropped (Sec. IV.D): the used symbols, in declaration
    order, become variables 0 .. N-1.  Integer coefficients give an integer
    tensor, otherwise real."""
    p = Poly._lift(expr)
    used = p.symbols()
    if not used:
        raise ValueError("the expression uses no symbol")
    col = {s: j for j, s in enumerate(used)}
    terms = [(k, v) for k, v in p.t.items()]
    integer = all(isinstance(v, int) for _, v in terms)
    ptr, idx, co = [0], [], []
    for k, v in terms:
        idx.extend(col[i] for i in k)
        ptr.append(len(idx))
        co.append(v)
    coeff = np.array(co, dtype=np.int64 if integer else np.float64)
    t = hobo.Tensor(len(used), np.array(ptr, dtype=np.int64), np.array(idx, dtype=np.int32), coeff,
                    max_order=max_order)
    return Compiled(tensor=t, offset=t.offset, symbol_ids=used, names=[_NAMES[i] for i in used])


@dataclass
class Sample:
    """One row of a sampling result: a distinct state, its energy (offset
    excluded, as the paper prints it) and how many samples ended in it."""
    bits: np.ndarray          # uint8 [N], variable order of the compiled tensor
    energy: object
    occurrence: int
    compiled: Compiled = field(repr=False)

    def by_id(self) -> dict:
        return {s: int(b) for s, b in zip(self.compiled.symbol_ids, self.bits)}

    def by_name(self) -> dict:
        return {n: int(b) for n, b in zip(self.compiled.names, self.bits)}

    def value(self, expr) -> float | int:
        """Value of an expression (e.g. an encoded integer) at this state."""
        return Poly._lift(expr).value(self.by_id())

    def array(self, fmt: str) -> tuple[np.ndarray, list]:
        """The symbols named by `fmt` (e.g. 'q{}_{}') as an integer array
        indexed like their names, with the sorted index tuples found; symbols
        compiled away are 0."""
        rx = re.compile("^" + re.escape(fmt).replace(r"\{\}", r"(-?\d+)") + "$")
        found = {}
        for name in _NAMES:
            m = rx.match(name)
            if m:
                found[tuple(int(g) for g in m.groups())] = name
        if not found:
            raise ValueError(f"no symbol matches {fmt!r}")
        subs = sorted(found)
        shape = tuple(max(s[d] for s in subs) + 1 for d in range(len(subs[0])))
        vals = self.by_name()
        out = np.zeros(shape, dtype=np.int64)
        for s in subs:
            out[s] = vals.get(found[s], 0)
        return out, subs


def sample(compiled: Compiled, shots: int, sweeps: int = 1000, t_start: float = 5.0, t_end: float = 0.01,
           seed: int = 0, precision: int | None = None) -> list[Sample]:
    """Anneal `shots` replicas (batched Metropolis, hobo_anneal_batch, one
    GPU), take each replica's best state with its exact energy, and return
    the distinct states best first with their occurrence counts
    (hobo_aggregate)."""
    import torch

    t = compiled.tensor
    W = (t.n_vars + 63) // 64
    dev = torch.device("cuda")
    x = torch.zeros(W * shots, dtype=torch.int64, device=dev)
    bx = torch.zeros_like(x)
    be = torch.zeros(shots, dtype=torch.int64 if t.integer else torch.float64, device=dev)
    kw = dict(sweeps=sweeps, t_start=t_start, t_end=t_end, seed=seed, init=hobo.INIT_RANDOM)
    if precision is not None:
        hobo.anneal_batch(t, shots, x, bx, be, precision=precision, **kw)
    else:
        # FP32 (exact for integer tensors whose sum |w| < 2^24), else INT8X4 digits
        try:
            hobo.anneal_batch(t, shots, x, bx, be, precision=hobo.PREC_FP32, **kw)
        except hobo.HoboError as e:
            if not (t.integer and e.code == hobo.ERR_RANGE):
                raise
            hobo.anneal_batch(t, shots, x, bx, be, precision=hobo.PREC_INT8X4, **kw)
    torch.cuda.synchronize()
    bits = hobo.bits_to_host(bx).reshape(W, shots)
    e = be.cpu().numpy()
    rep, cnt = hobo.aggregate(t.n_vars, bits, e)
    rows = []
    for r, c in zip(rep, cnt):
        b = np.array([(int(bits[i >> 6, r]) >> (i & 63)) & 1 for i in range(t.n_vars)], dtype=np.uint8)
        rows.append(Sample(bits=b, energy=int(e[r]) if t.integer else float(e[r]), occurrence=int(c),
                           compiled=compiled))
    return rows

