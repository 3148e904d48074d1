"""Training data, training and evaluation of the learned flip proposal,
driven entirely through the C-ABI (every computation runs in the library's
kernels; this module only orders the calls and holds device buffers).

* :func:`record_transitions` (hobo_record_transitions) runs a plain
  annealing schedule; before each recorded sweep the fields of the current
  states give every bit's features [x_i, beta_s dE_i, beta_s ||H_i||]; after
  the sweep its label is whether the bit changed.
* :func:`train` fits the 3 -> 256 -> 1 network on those transitions
  (hobo_mlp_train: BCE, Adam, deterministic sums).
* :func:`anneal_timed` runs one annealing call (plain or LEARNED) and returns
  its kernel time, best energies and per-sweep trace.
"""
from __future__ import annotations

import numpy as np

from . import hobo


def record_transitions(t: "hobo.Tensor", replicas: int, sweeps: int, t_start: float, t_end: float, seed: int,
                       record: list, precision: int = hobo.PREC_BF16X2):
    """Transitions of a plain annealing run (hobo_record_transitions): for
    each sweep index in ``record``, the features of every (replica, bit) at
    the sweep's start and the label "the bit changed during the sweep".
    Returns device tensors (feats [M][3], labels [M]) with
    M = len(record) * replicas * N."""
    import torch

    n, b = t.n_vars, int(replicas)
    rec = sorted(set(int(s) for s in record if 0 <= int(s) < sweeps))
    feats = torch.empty((len(rec), b, n, 3), dtype=torch.float32, device="cuda")
    labels = torch.empty((len(rec), b, n), dtype=torch.float32, device="cuda")
    hobo.record_transitions(t, b, rec, feats, labels, sweeps=sweeps, t_start=t_start, t_end=t_end, seed=seed,
                            precision=precision)
    return feats.reshape(-1, 3).contiguous(), labels.reshape(-1).contiguous()


def train(feats, labels, params0: np.ndarray, *, batch: int = 4096, epochs: int = 3, lr: float = 1e-3):
    """Trains from ``params0`` (FP32 [1281]); returns (state [3*1284] device
    FP32 whose first 1281 values are the parameters, loss per step)."""
    import torch

    st = torch.zeros(hobo.MLP_STATE, dtype=torch.float32, device="cuda")
    st[:hobo.MLP_PARAMS] = torch.from_numpy(np.ascontiguousarray(params0, dtype=np.float32)).cuda()
    m = labels.numel()
    steps = epochs * ((m + batch - 1) // batch)
    lt = torch.empty(max(steps, 1), dtype=torch.float32, device="cuda")
    hobo.mlp_train(st, feats, labels, batch=batch, epochs=epochs, lr=lr, loss_trace=lt)
    return st, lt[:steps]


def anneal_timed(t: "hobo.Tensor", replicas: int, sweeps: int, t_start: float, t_end: float, seed: int, *,
                 precision: int = hobo.PREC_BF16X2, mlp=None, tau: float = 0.5, p_floor: float = 0.0,
                 refresh: int = 10, repeats: int = 1, algorithm: int = hobo.ANNEAL_AUTO):
    """One annealing call (LEARNED when ``mlp`` is given) timed with HIP
    events around the call on the current stream; returns dict(ms, best_e,
    trace) of the last repeat."""
    import torch

    n, b = t.n_vars, int(replicas)
    w = (n + 63) // 64
    x = torch.zeros(w * b, dtype=torch.int64, device="cuda")
    bx = torch.zeros_like(x)
    be = torch.zeros(b, dtype=torch.int64 if t.integer else torch.float64, device="cuda")
    tr = torch.zeros(max(sweeps, 1), dtype=torch.float64, device="cuda")
    kw = dict(sweeps=sweeps, t_start=t_start, t_end=t_end, seed=seed, precision=precision, trace_out=tr,
              algorithm=algorithm)
    if mlp is not None:
        kw.update(mlp=mlp, tau=tau, p_floor=p_floor, refresh=refresh)
    hobo.anneal_batch(t, b, x, bx, be, **kw)  # warm-up: layouts and cached setup
    torch.cuda.synchronize()
    ms = []
    for _ in range(repeats):
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        hobo.anneal_batch(t, b, x, bx, be, **kw)
        z.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(z))
    return dict(ms=float(np.median(ms)), best_e=be.cpu().numpy(), trace=tr.cpu().numpy()[:sweeps])
