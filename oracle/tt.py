"""Oracle for the tensor-train (TT) form of the HOBO tensor (Sec. VI.E-F).

Test infrastructure, like the rest of oracle/: only the tests, the smoke
entry point and the benchmark's CPU-baseline leg use it.

* tt_svd: the paper's sequential TT decomposition without approximation --
  reshape the tensor into a matrix, take its SVD, keep the left factor as
  the core, carry Sigma V* into the next step and repeat (Sec. VI.E), with
  numpy's SVD as the library step and singular values kept where
  sigma > sigma_max * max(rows, cols) * eps (numpy's numerical-rank rule).
* tt_energies: E(x) = sum H_{i1..id} x_{i1} .. x_{id} evaluated through the
  cores, E = prod_k (sum_i x_i G_k[:, i, :]) (the TT form of the batch
  contraction of Sec. IV.C), in FP64.
* tt_full: the dense tensor the cores represent.
"""
from __future__ import annotations

import numpy as np


def tt_svd(h: np.ndarray):
    """Cores G_k of shape (r_{k-1}, n_k, r_k), r_0 = r_d = 1, and the ranks
    [r_1 .. r_{d-1}]."""
    h = np.asarray(h, dtype=np.float64)
    dims = h.shape
    d = len(dims)
    cores, ranks = [], []
    c = h.reshape(dims[0], -1)
    r_prev = 1
    for k in range(d - 1):
        c = c.reshape(r_prev * dims[k], -1)
        u, s, vt = np.linalg.svd(c, full_matrices=False)
        tol = s.max(initial=0.0) * max(c.shape) * np.finfo(np.float64).eps
        r = max(int(np.count_nonzero(s > tol)), 1)
        cores.append(u[:, :r].reshape(r_prev, dims[k], r))
        c = s[:r, None] * vt[:r, :]
        ranks.append(r)
        r_prev = r
    cores.append(c.reshape(r_prev, dims[-1], 1))
    return cores, ranks


def tt_full(cores) -> np.ndarray:
    """The dense tensor of a core list (contracted one bond at a time)."""
    t = cores[0]
    for g in cores[1:]:
        t = np.tensordot(t, g, axes=([t.ndim - 1], [0]))
    return t.reshape(t.shape[1:-1])


def tt_energies(cores, x_rows: np.ndarray) -> np.ndarray:
    """E_b = prod over cores of (sum_i x_{b,i} G_k[:, i, :]) for each row."""
    x = np.asarray(x_rows, dtype=np.float64)
    out = np.empty(x.shape[0])
    for b, row in enumerate(x):
        v = np.ones((1,))
        for g in cores:
            v = v @ np.tensordot(row, g, axes=([0], [1]))  # (r_{k-1}, r_k) matrix of this row
        out[b] = v[0]
    return out
