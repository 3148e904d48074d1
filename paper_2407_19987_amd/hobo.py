"""Python binding of the HOBO engine's C-ABI (include/hobo.h).

Argument marshalling only: every computation runs in libhobo.so's HIP
kernels.  PyTorch supplies device memory and streams.  Importing this module
raises if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
# torch (the device-memory and stream provider) is loaded before the library:
# the library then binds to the HIP runtime torch already holds, and both see
# the same devices whatever the import order of the caller
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhobo.so")

# status codes
OK, ERR_INVALID_ARG, ERR_ORDER, ERR_RANGE, ERR_PRECISION, ERR_NO_DEVICE, ERR_OOM, ERR_HIP, ERR_UNSUPPORTED = range(9)
COEFF_INT64, COEFF_F64 = 0, 1
PREC_FP32, PREC_BF16X2, PREC_BF16X3, PREC_INT8X4, PREC_FP64, PREC_FP16X2 = range(6)
PREC_NAMES = {"fp32": PREC_FP32, "bf16x2": PREC_BF16X2, "bf16x3": PREC_BF16X3, "int8x4": PREC_INT8X4,
              "fp64": PREC_FP64, "fp16x2": PREC_FP16X2}
INIT_RANDOM, INIT_GIVEN = 0, 1
PROPOSAL_METROPOLIS, PROPOSAL_MASKED, PROPOSAL_LEARNED = 0, 1, 2
ANNEAL_AUTO, ANNEAL_SLABS, ANNEAL_BLOCKS = 0, 1, 2
LAUNCH_PER_INSTANCE, LAUNCH_PERSISTENT, LAUNCH_GRAPH = 0, 1, 2
FN_ENERGY, FN_FIELDS, FN_ANNEAL = 1, 2, 4
MLP_HIDDEN, MLP_FEATURES = 256, 3
MLP_PARAMS = MLP_FEATURES * MLP_HIDDEN + 2 * MLP_HIDDEN + 1
MLP_ROW = 1284
MLP_STATE = 3 * MLP_ROW

EXPORTS = [
    "hobo_build_tensor", "hobo_free_tensor", "hobo_tensor_info_get", "hobo_tensor_monomials",
    "hobo_tensor_export_dense", "hobo_tensor_prepare", "hobo_energy", "hobo_local_fields",
    "hobo_anneal_batch", "hobo_timing_enable", "hobo_timing_read", "hobo_last_error", "hobo_version",
    "hobo_mlp_forward", "hobo_mlp_grad", "hobo_mlp_train", "hobo_proposal_features", "hobo_autotune",
    "hobo_tensor_layout_info", "hobo_energy_noalloc", "hobo_aggregate",
    "hobo_tt_build", "hobo_tt_free", "hobo_tt_info", "hobo_tt_cores", "hobo_tt_energy",
    "hobo_gd_gradient", "hobo_gd_batch", "hobo_record_transitions",
]


class HoboError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hobo status {code}: {msg}")
        self.code = code


class TensorInfo(ctypes.Structure):
    _fields_ = [("n_vars", ctypes.c_int32), ("order", ctypes.c_int32), ("is_integer", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n_monomials", ctypes.c_int64), ("n_per_order", ctypes.c_int64 * 8),
                ("offset_i64", ctypes.c_int64), ("offset_f64", ctypes.c_double), ("device_bytes", ctypes.c_int64)]


class LayoutInfo(ctypes.Structure):
    _fields_ = [("chunks", ctypes.c_int64), ("tiles", ctypes.c_int64), ("issued_flops", ctypes.c_int64),
                ("bytes", ctypes.c_int64)]


class AnnealParams(ctypes.Structure):
    _fields_ = [("sweeps", ctypes.c_int32), ("precision", ctypes.c_int32), ("t_start", ctypes.c_double),
                ("t_end", ctypes.c_double), ("seed", ctypes.c_uint64), ("init", ctypes.c_int32),
                ("proposal", ctypes.c_int32), ("attempt", ctypes.c_void_p), ("waves_per_block", ctypes.c_int32),
                ("algorithm", ctypes.c_int32), ("first_sweep", ctypes.c_int32), ("schedule_sweeps", ctypes.c_int32),
                ("continue_best", ctypes.c_int32), ("refresh", ctypes.c_int32), ("mlp", ctypes.c_void_p),
                ("tau", ctypes.c_float), ("p_floor", ctypes.c_float)]


class GDParams(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("init", ctypes.c_int32), ("eta", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class MlpTrainParams(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("epochs", ctypes.c_int32), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("step0", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2407_19987_amd.build` first")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    lib.hobo_build_tensor.argtypes = [i32, i32, i64, P, P, P, i32, ctypes.POINTER(P), P]
    lib.hobo_free_tensor.argtypes = [P]
    lib.hobo_tensor_info_get.argtypes = [P, ctypes.POINTER(TensorInfo)]
    lib.hobo_tensor_monomials.argtypes = [P, P, i64, P, i64, P, i64]
    lib.hobo_tensor_export_dense.argtypes = [P, P, i64]
    lib.hobo_tensor_prepare.argtypes = [P, u32, u32]
    lib.hobo_tensor_layout_info.argtypes = [P, i32, i32, ctypes.POINTER(LayoutInfo)]
    lib.hobo_energy.argtypes = [P, P, i64, i32, P, P]
    lib.hobo_energy_noalloc.argtypes = [P, P, i64, i32, P, P]
    lib.hobo_aggregate.argtypes = [i32, i64, P, P, i32, P, P, P]
    lib.hobo_tt_build.argtypes = [P, ctypes.POINTER(P)]
    lib.hobo_tt_free.argtypes = [P]
    lib.hobo_tt_info.argtypes = [P, P, P, P, P]
    lib.hobo_tt_cores.argtypes = [P, P, i64]
    lib.hobo_tt_energy.argtypes = [P, P, i64, P, P]
    lib.hobo_gd_gradient.argtypes = [P, P, i64, P, P]
    lib.hobo_record_transitions.argtypes = [P, i64, ctypes.POINTER(AnnealParams), P, i32, P, P, P]
    lib.hobo_gd_batch.argtypes = [P, i64, ctypes.POINTER(GDParams), P, P, P, P]
    lib.hobo_local_fields.argtypes = [P, P, i64, i32, P, P, P]
    lib.hobo_anneal_batch.argtypes = [P, i32, P, ctypes.POINTER(AnnealParams), P, P, P, P, i32, P]
    lib.hobo_mlp_forward.argtypes = [P, P, i64, P, P]
    lib.hobo_mlp_grad.argtypes = [P, P, P, i64, P, P, P]
    lib.hobo_autotune.argtypes = [P, P, i64, i32, i32, P, P]
    lib.hobo_mlp_train.argtypes = [P, P, P, i64, ctypes.POINTER(MlpTrainParams), P, P]
    lib.hobo_proposal_features.argtypes = [P, P, P, i64, P, ctypes.c_double, ctypes.c_double, i32, i32, P, P, P]
    lib.hobo_timing_enable.argtypes = [i32]
    lib.hobo_timing_read.argtypes = [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    for name in EXPORTS:
        if name in ("hobo_last_error", "hobo_version"):
            getattr(lib, name).restype = ctypes.c_char_p
            getattr(lib, name).argtypes = []
        else:
            getattr(lib, name).restype = i32
    return lib


lib = _load()


def _check(code: int):
    if code != OK:
        raise HoboError(code, lib.hobo_last_error().decode())


def version() -> str:
    return lib.hobo_version().decode()


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Tensor:
    """Owning handle of a compiled HOBO instance (hobo_build_tensor)."""

    def __init__(self, n_vars: int, term_ptr, term_idx, coeff, max_order: int = 0):
        tp = np.ascontiguousarray(term_ptr, dtype=np.int64)
        ti = np.ascontiguousarray(term_idx, dtype=np.int32)
        co = np.asarray(coeff)
        integer = co.dtype.kind in "iu"
        co = np.ascontiguousarray(co, dtype=np.int64 if integer else np.float64)
        h = ctypes.c_void_p()
        off = np.zeros(1, dtype=np.int64 if integer else np.float64)
        _check(lib.hobo_build_tensor(int(n_vars), int(max_order), len(co), _np_ptr(tp), _np_ptr(ti), _np_ptr(co),
                                     COEFF_INT64 if integer else COEFF_F64, ctypes.byref(h), _np_ptr(off)))
        self._h = h
        self.integer = integer
        self.offset = int(off[0]) if integer else float(off[0])
        info = self.info()
        self.n_vars = info.n_vars
        self.order = info.order
        self.n_monomials = info.n_monomials

    @classmethod
    def from_terms(cls, terms, max_order: int = 0) -> "Tensor":
        return cls(terms.n_vars, terms.term_ptr, terms.term_idx, terms.coeff, max_order)

    @property
    def handle(self):
        return self._h

    def info(self) -> TensorInfo:
        inf = TensorInfo()
        _check(lib.hobo_tensor_info_get(self._h, ctypes.byref(inf)))
        return inf

    def monomials(self):
        n = self.info().n_monomials
        ptr = np.zeros(n + 1, dtype=np.int64)
        _check(lib.hobo_tensor_monomials(self._h, _np_ptr(ptr), n + 1, None, 0, None, 0))
        idx = np.zeros(max(int(ptr[-1]), 1), dtype=np.int32)
        w = np.zeros(max(n, 1), dtype=np.int64 if self.integer else np.float64)
        _check(lib.hobo_tensor_monomials(self._h, None, 0, _np_ptr(idx), len(idx), _np_ptr(w), len(w)))
        return ptr, idx[: int(ptr[-1])], w[:n]

    def export_dense(self) -> np.ndarray:
        k = max(self.order, 1)
        out = np.zeros(self.n_vars ** k, dtype=np.int64 if self.integer else np.float64)
        _check(lib.hobo_tensor_export_dense(self._h, _np_ptr(out), out.size))
        return out.reshape((self.n_vars,) * k)

    def prepare(self, fn_mask: int, prec_mask: int):
        _check(lib.hobo_tensor_prepare(self._h, fn_mask, prec_mask))

    def layout_info(self, fn: int, precision: int) -> LayoutInfo:
        inf = LayoutInfo()
        _check(lib.hobo_tensor_layout_info(self._h, int(fn), int(precision), ctypes.byref(inf)))
        return inf

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.hobo_free_tensor(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ device calls


def _dev_ptr(t) -> int:
    import torch

    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


def _stream(stream) -> int:
    import torch

    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _check_bits(t: Tensor, x_bits, B: int):
    w = (t.n_vars + 63) // 64
    if x_bits.numel() < w * B or x_bits.element_size() != 8:
        raise ValueError("x_bits must hold [W][B] 64-bit words")


def energy(t: Tensor, x_bits, B: int, precision: int, e_out, stream=None):
    """hobo_energy: e_out (int64 for integer tensors, float64 otherwise) [B]."""
    _check_bits(t, x_bits, B)
    if e_out.numel() < B or e_out.element_size() != 8:
        raise ValueError("e_out must hold B 8-byte values")
    _check(lib.hobo_energy(t.handle, _dev_ptr(x_bits), int(B), int(precision), _dev_ptr(e_out), _stream(stream)))


def energy_noalloc(t: Tensor, x_bits, B: int, precision: int, e_out, stream=None):
    """hobo_energy_noalloc: as energy(), with the library's per-GPU scratch
    instead of any allocation (the layout must be prepared first)."""
    _check_bits(t, x_bits, B)
    if e_out.numel() < B or e_out.element_size() != 8:
        raise ValueError("e_out must hold B 8-byte values")
    _check(lib.hobo_energy_noalloc(t.handle, _dev_ptr(x_bits), int(B), int(precision), _dev_ptr(e_out),
                                   _stream(stream)))


def local_fields(t: Tensor, x_bits, B: int, precision: int, de_out, e_out=None, stream=None):
    """hobo_local_fields: de_out [B][N] (int64 for integer tensors, float32 otherwise)."""
    _check_bits(t, x_bits, B)
    want = 8 if t.integer else 4
    if de_out.numel() < B * t.n_vars or de_out.element_size() != want:
        raise ValueError("de_out has the wrong size or dtype")
    ep = None
    if e_out is not None:
        if e_out.numel() < B or e_out.element_size() != 8:
            raise ValueError("e_out must hold B 8-byte values")
        ep = _dev_ptr(e_out)
    _check(lib.hobo_local_fields(t.handle, _dev_ptr(x_bits), int(B), int(precision), _dev_ptr(de_out), ep,
                                 _stream(stream)))


def anneal_batch(tensors, replicas, x_inout, best_x_out, best_e_out, *, sweeps: int, t_start: float, t_end: float,
                 seed: int, precision: int = PREC_FP32, init: int = INIT_RANDOM, attempt=None, trace_out=None,
                 launch_mode: int = LAUNCH_PERSISTENT, waves_per_block: int = 0, algorithm: int = ANNEAL_AUTO,
                 first_sweep: int = 0, schedule_sweeps: int = 0, continue_best: bool = False, mlp=None,
                 tau: float = 0.5, p_floor: float = 0.0, refresh: int = 1, stream=None):
    """hobo_anneal_batch over one or several instances (concatenated buffers).
    ``attempt`` selects MASKED, ``mlp`` (device FP32 parameters) LEARNED."""
    if isinstance(tensors, Tensor):
        tensors = [tensors]
    n = len(tensors)
    reps = np.ascontiguousarray(replicas if np.ndim(replicas) else [replicas], dtype=np.int64)
    if len(reps) != n:
        raise ValueError("one replica count per tensor")
    words = sum(((t.n_vars + 63) // 64) * int(b) for t, b in zip(tensors, reps))
    if x_inout.numel() < words or best_x_out.numel() < words:
        raise ValueError("bit buffers too small")
    if best_e_out.numel() < int(reps.sum()) or best_e_out.element_size() != 8:
        raise ValueError("best_e_out too small")
    if trace_out is not None and trace_out.numel() < n * sweeps:
        raise ValueError("trace_out too small")
    if attempt is not None:
        need = sum(((int(b) + 15) // 16) * int(sweeps) * t.n_vars for t, b in zip(tensors, reps))
        if attempt.numel() < need or attempt.element_size() != 1:
            raise ValueError(f"attempt masks must hold {need} bytes")
    if mlp is not None and (mlp.numel() < MLP_PARAMS or mlp.element_size() != 4):
        raise ValueError(f"mlp must hold {MLP_PARAMS} FP32 values")
    handles = (ctypes.c_void_p * n)(*[t.handle.value for t in tensors])
    p = AnnealParams()
    p.sweeps = int(sweeps)
    p.precision = int(precision)
    p.t_start = float(t_start)
    p.t_end = float(t_end)
    p.seed = int(seed)
    p.init = int(init)
    p.proposal = PROPOSAL_MASKED if attempt is not None else (PROPOSAL_LEARNED if mlp is not None else
                                                               PROPOSAL_METROPOLIS)
    p.attempt = _dev_ptr(attempt) if attempt is not None else None
    p.waves_per_block = int(waves_per_block)
    p.algorithm = int(algorithm)
    p.first_sweep = int(first_sweep)
    p.schedule_sweeps = int(schedule_sweeps)
    p.continue_best = 1 if continue_best else 0
    p.refresh = int(refresh)
    p.mlp = _dev_ptr(mlp) if mlp is not None else None
    p.tau = float(tau)
    p.p_floor = float(p_floor)
    _check(lib.hobo_anneal_batch(handles, n, _np_ptr(reps), ctypes.byref(p), _dev_ptr(x_inout), _dev_ptr(best_x_out),
                                 _dev_ptr(best_e_out), _dev_ptr(trace_out) if trace_out is not None else None,
                                 int(launch_mode), _stream(stream)))


def mlp_forward(params, feats, logits_out, stream=None):
    """hobo_mlp_forward: logits of feats [M][3] (device FP32)."""
    m = feats.numel() // 3
    if feats.numel() != 3 * m or logits_out.numel() < m or params.numel() < MLP_PARAMS:
        raise ValueError("feats must be [M][3], logits_out [M], params [1281]")
    _check(lib.hobo_mlp_forward(_dev_ptr(params), _dev_ptr(feats), m, _dev_ptr(logits_out), _stream(stream)))


def mlp_grad(params, feats, labels, grad_out, loss_out=None, stream=None):
    """hobo_mlp_grad: mean-BCE gradient over all samples (device FP32)."""
    m = feats.numel() // 3
    if feats.numel() != 3 * m or labels.numel() < m or grad_out.numel() < MLP_PARAMS:
        raise ValueError("feats must be [M][3], labels [M], grad_out [1281]")
    _check(lib.hobo_mlp_grad(_dev_ptr(params), _dev_ptr(feats), _dev_ptr(labels), m, _dev_ptr(grad_out),
                             _dev_ptr(loss_out) if loss_out is not None else None, _stream(stream)))


def mlp_train(state, feats, labels, *, batch: int, epochs: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8, step0: int = 0, loss_trace=None, stream=None):
    """hobo_mlp_train on a device FP32 state [params | m | v] (rows of 1284)."""
    m = feats.numel() // 3
    if feats.numel() != 3 * m or labels.numel() < m or state.numel() < MLP_STATE:
        raise ValueError("feats must be [M][3], labels [M], state [3 * 1284]")
    steps = epochs * ((m + batch - 1) // batch)
    if loss_trace is not None and loss_trace.numel() < steps:
        raise ValueError(f"loss_trace must hold {steps} values")
    tp = MlpTrainParams(int(batch), int(epochs), float(lr), float(beta1), float(beta2), float(eps), int(step0))
    _check(lib.hobo_mlp_train(_dev_ptr(state), _dev_ptr(feats), _dev_ptr(labels), m, ctypes.byref(tp),
                              _dev_ptr(loss_trace) if loss_trace is not None else None, _stream(stream)))


def proposal_features(t: Tensor, x_bits, B: int, de, feats_out, *, t_start: float, t_end: float, sweep: int,
                      schedule_sweeps: int, x_after=None, labels_out=None, stream=None):
    """hobo_proposal_features: feats_out [B][N][3] before sweep `sweep` of the
    schedule (and transition labels)."""
    _check_bits(t, x_bits, B)
    n = t.n_vars
    if feats_out.numel() < 3 * B * n or de.numel() < B * n:
        raise ValueError("feats_out must hold B*N*3 values and de B*N")
    if labels_out is not None and (x_after is None or labels_out.numel() < B * n):
        raise ValueError("labels need x_after and B*N values")
    _check(lib.hobo_proposal_features(t.handle, _dev_ptr(x_bits), _dev_ptr(x_after) if x_after is not None else None,
                                      int(B), _dev_ptr(de), float(t_start), float(t_end), int(sweep),
                                      int(schedule_sweeps), _dev_ptr(feats_out),
                                      _dev_ptr(labels_out) if labels_out is not None else None, _stream(stream)))


def autotune(t: Tensor, x_bits, B: int, fn_mask: int, precision: int, stream=None):
    """hobo_autotune: returns the chosen shapes (energy, fields, anneal)."""
    _check_bits(t, x_bits, B)
    out = np.zeros(3, dtype=np.int32)
    _check(lib.hobo_autotune(t.handle, _dev_ptr(x_bits), int(B), int(fn_mask), int(precision), _np_ptr(out),
                             _stream(stream)))
    return tuple(int(v) for v in out)


KERNEL_ANNEAL, KERNEL_FIELDS, KERNEL_ENERGY = 0, 1, 2


def timing_enable(on: bool = True):
    _check(lib.hobo_timing_enable(1 if on else 0))


def timing_read(kernel: int):
    """(total milliseconds, launches) of the timed launches of one kernel."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib.hobo_timing_read(int(kernel), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def bits_to_device(bits_np: np.ndarray):
    """numpy uint64 [W][B] -> torch int64 device tensor with the same bytes."""
    import torch

    return torch.from_numpy(np.ascontiguousarray(bits_np, dtype=np.uint64).view(np.int64)).cuda()


def bits_to_host(bits_dev) -> np.ndarray:
    return bits_dev.cpu().numpy().view(np.uint64)


def aggregate(n_vars: int, bits_host: np.ndarray, energies_host: np.ndarray):
    """hobo_aggregate on host arrays: bits [W][B] uint64, energies [B] int64 or
    float64.  Returns (representative sample index [U], count [U]), best first."""
    bits = np.ascontiguousarray(bits_host, dtype=np.uint64)
    e = np.ascontiguousarray(energies_host)
    integer = e.dtype.kind in "iu"
    e = np.ascontiguousarray(e, dtype=np.int64 if integer else np.float64)
    B = e.shape[0]
    if bits.shape != ((n_vars + 63) // 64, B):
        raise ValueError("bits must be [W][B]")
    rep = np.zeros(max(B, 1), dtype=np.int64)
    cnt = np.zeros(max(B, 1), dtype=np.int64)
    nu = np.zeros(1, dtype=np.int64)
    _check(lib.hobo_aggregate(int(n_vars), int(B), _np_ptr(bits), _np_ptr(e), 1 if integer else 0, _np_ptr(nu),
                              _np_ptr(rep), _np_ptr(cnt)))
    u = int(nu[0])
    return rep[:u], cnt[:u]


class TensorTrain:
    """Owning handle of the TT form of a tensor (hobo_tt_build)."""

    def __init__(self, t: Tensor):
        h = ctypes.c_void_p()
        _check(lib.hobo_tt_build(t.handle, ctypes.byref(h)))
        self._h = h
        order, n = np.zeros(1, np.int32), np.zeros(1, np.int32)
        ranks = np.zeros(9, np.int32)
        npar = np.zeros(1, np.int64)
        _check(lib.hobo_tt_info(h, _np_ptr(order), _np_ptr(n), _np_ptr(ranks), _np_ptr(npar)))
        self.order, self.n_vars = int(order[0]), int(n[0])
        self.ranks = [int(r) for r in ranks[: self.order + 1]]
        self.n_params = int(npar[0])

    def cores(self) -> list:
        flat = np.zeros(max(self.n_params, 1), dtype=np.float64)
        _check(lib.hobo_tt_cores(self._h, _np_ptr(flat), len(flat)))
        out, off = [], 0
        for k in range(self.order):
            shape = (self.ranks[k], self.n_vars, self.ranks[k + 1])
            size = int(np.prod(shape))
            out.append(flat[off:off + size].reshape(shape))
            off += size
        return out

    def energy(self, x_bits, B: int, e_out, stream=None):
        w = (self.n_vars + 63) // 64
        if x_bits.numel() < w * B or e_out.numel() < B or e_out.element_size() != 8:
            raise ValueError("x_bits [W][B] words and e_out [B] doubles")
        _check(lib.hobo_tt_energy(self._h, _dev_ptr(x_bits), int(B), _dev_ptr(e_out), _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.hobo_tt_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gd_gradient(t: Tensor, p, B: int, g_out, stream=None):
    """hobo_gd_gradient: p, g_out device float64 [N][B]."""
    if p.numel() < t.n_vars * B or g_out.numel() < t.n_vars * B or p.element_size() != 8:
        raise ValueError("p and g_out must hold [N][B] doubles")
    _check(lib.hobo_gd_gradient(t.handle, _dev_ptr(p), int(B), _dev_ptr(g_out), _stream(stream)))


def gd_batch(t: Tensor, B: int, p_inout, x_out, e_out, *, iterations: int, eta: float, seed: int = 0,
             init: int = INIT_RANDOM, stream=None):
    """hobo_gd_batch: p_inout device float64 [N][B], x_out [W][B] words, e_out [B]."""
    w = (t.n_vars + 63) // 64
    if p_inout.numel() < t.n_vars * B or x_out.numel() < w * B or e_out.numel() < B:
        raise ValueError("buffer sizes")
    prm = GDParams(int(iterations), int(init), float(eta), int(seed))
    _check(lib.hobo_gd_batch(t.handle, int(B), ctypes.byref(prm), _dev_ptr(p_inout), _dev_ptr(x_out),
                             _dev_ptr(e_out), _stream(stream)))


def record_transitions(t: Tensor, B: int, record, feats_out, labels_out, *, sweeps: int, t_start: float, t_end: float,
                       seed: int, precision: int = PREC_FP32, init: int = INIT_RANDOM, stream=None):
    """hobo_record_transitions: features before and labels of the sweeps in
    `record` of a plain run; feats_out [len(record)][B][N][3], labels_out
    [len(record)][B][N] device FP32."""
    rec = np.ascontiguousarray(sorted(set(int(r) for r in record)), dtype=np.int32)
    n = t.n_vars
    if feats_out.numel() < len(rec) * B * n * 3 or labels_out.numel() < len(rec) * B * n:
        raise ValueError("feats_out / labels_out too small")
    p = AnnealParams()
    p.sweeps, p.precision, p.t_start, p.t_end, p.seed = int(sweeps), int(precision), float(t_start), float(t_end), \
        int(seed)
    p.init, p.proposal = int(init), PROPOSAL_METROPOLIS
    _check(lib.hobo_record_transitions(t.handle, int(B), ctypes.byref(p), _np_ptr(rec), len(rec),
                                       _dev_ptr(feats_out), _dev_ptr(labels_out), _stream(stream)))
