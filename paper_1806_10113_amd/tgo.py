"""Python binding of libtgo.so: argument marshalling only.

Device memory and streams come from PyTorch (ROCm); every step of the model
runs in the library's HIP kernels.  If the library is missing this module
raises at the first call: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# TGO_LIB names another build of the same sources (the host-sanitizer test
# loads one this way); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("TGO_LIB") or os.path.join(_PKG, "libtgo.so")

TGO_OK, TGO_EINVAL, TGO_ERANGE, TGO_ENOMEM, TGO_EDEVICE = 0, -1, -2, -3, -4
MAX_N = 16
MAX_EXHAUSTIVE_N = 13


class TgoError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: error {code} ({detail})")
        self.code = code


class _Model(ctypes.Structure):
    _fields_ = [("dma_engines", ctypes.c_int32), ("q_log2", ctypes.c_int32),
                ("p_htd", ctypes.c_int32), ("p_dth", ctypes.c_int32)]


SUMMARY_DTYPE = np.dtype([
    ("min_ns", "<i8"), ("max_ns", "<i8"), ("argmin_rank", "<u8"), ("argmax_rank", "<u8"),
    ("sum_lo", "<u8"), ("sum_hi", "<u8"), ("count", "<u8"), ("fingerprint", "<u8"),
    ("mean_ns", "<f8"), ("status", "<i4"), ("n", "<i4"), ("best", "u1", (16,)),
    ("worst", "u1", (16,)), ("heur", "u1", (16,)), ("heur_ns", "<i8"),
])
assert SUMMARY_DTYPE.itemsize == 136


@dataclass(frozen=True)
class Model:
    """Overlapped HtD/DtH advance at p_htd/q and p_dth/q of solo speed, q = 2**q_log2."""

    q_log2: int = 2
    p_htd: int = 3
    p_dth: int = 3
    dma_engines: int = 2

    @property
    def q(self) -> int:
        return 1 << self.q_log2

    def _c(self) -> _Model:
        return _Model(self.dma_engines, self.q_log2, self.p_htd, self.p_dth)


DEFAULT = Model(2, 3, 3)
PAPER_EXAMPLE = Model(3, 3, 3)
NO_SLOWDOWN = Model(0, 1, 1)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_1806_10113_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        M = ctypes.POINTER(_Model)
        L.tgo_strerror.restype = ctypes.c_char_p
        L.tgo_strerror.argtypes = [i32]
        L.tgo_last_error.restype = ctypes.c_char_p
        L.tgo_last_error.argtypes = []
        L.tgo_version.restype = i32
        L.tgo_evaluate.argtypes = [M, vp, i32, vp, i64, vp, vp]
        L.tgo_exhaustive.argtypes = [M, vp, i32, vp, vp, vp]
        L.tgo_exhaustive_noalloc.argtypes = [M, vp, i32, vp, vp, vp]
        L.tgo_exhaustive_noalloc.restype = i32
        L.tgo_heuristic.argtypes = [M, vp, vp, i32, vp, vp, vp]
        L.tgo_rounds.argtypes = [M, vp, i32, i32, vp, vp, vp, vp]
        L.tgo_exhaustive_mem.argtypes = [M, vp, vp, i32, i64, vp, vp, vp]
        L.tgo_exhaustive_mem.restype = i32
        L.tgo_evaluate_mem.argtypes = [M, vp, vp, i32, i64, vp, i64, vp, vp]
        L.tgo_evaluate_mem.restype = i32
        L.tgo_predict.argtypes = [M, vp, i32, vp, ctypes.POINTER(ctypes.c_int64)]
        L.tgo_predict.restype = i32
        L.tgo_surrogate_save.argtypes = [vp, ctypes.c_char_p]
        L.tgo_surrogate_save.restype = i32
        L.tgo_surrogate_load.argtypes = [vp, ctypes.c_char_p]
        L.tgo_surrogate_load.restype = i32
        L.tgo_rank.argtypes = [i32, vp, ctypes.POINTER(ctypes.c_uint64)]
        L.tgo_unrank.argtypes = [i32, ctypes.c_uint64, vp]
        L.tgo_plan_create.argtypes = [M, i32, i32, ctypes.c_size_t, ctypes.POINTER(vp)]
        L.tgo_plan_autotune.argtypes = [vp, vp, vp, i32, vp, vp]
        L.tgo_plan_describe.argtypes = [vp, ctypes.c_char_p, ctypes.c_size_t]
        L.tgo_plan_set_decomposition.argtypes = [vp, vp, i32, i32]
        L.tgo_batch.argtypes = [vp, vp, vp, i32, vp, vp]
        L.tgo_surrogate_create.argtypes = [i64, i32, ctypes.POINTER(vp)]
        L.tgo_surrogate_destroy.argtypes = [vp]
        L.tgo_surrogate_destroy.restype = None
        L.tgo_surrogate_param_count.argtypes = []
        L.tgo_surrogate_init.argtypes = [vp, ctypes.c_uint64, vp]
        L.tgo_surrogate_set_params.argtypes = [vp, vp, vp]
        L.tgo_surrogate_get_params.argtypes = [vp, vp, vp]
        L.tgo_surrogate_pairs.argtypes = [M, vp, vp, i32, i64, ctypes.c_uint64, vp, vp, vp, vp, vp]
        L.tgo_surrogate_score.argtypes = [vp, vp, vp, i32, vp, vp, i64, vp, vp]
        L.tgo_surrogate_grad.argtypes = [vp, vp, vp, i32, vp, vp, vp, i32, vp, vp, vp]
        L.tgo_surrogate_train_step.argtypes = [vp, vp, vp, i32, vp, vp, vp, i32, ctypes.c_float, vp, vp]
        L.tgo_surrogate_search.argtypes = [vp, M, vp, vp, vp, i32, i64, i32, ctypes.c_uint64, vp, vp]
        L.tgo_random_search.argtypes = [M, vp, vp, i32, i64, ctypes.c_uint64, vp, vp]
        L.tgo_surrogate_candidates.argtypes = [vp, M, vp, vp, vp, i32, i64, i32, ctypes.c_uint64, vp, vp]
        L.tgo_surrogate_candidates.restype = i32
        L.tgo_exhaustive_cke.argtypes = [M, vp, vp, i32, i32, vp, vp, vp]
        L.tgo_exhaustive_cke.restype = i32
        L.tgo_evaluate_cke.argtypes = [M, vp, vp, i32, i32, vp, i64, vp, vp]
        L.tgo_evaluate_cke.restype = i32
        L.tgo_surrogate_adam_step.argtypes = [vp, vp, ctypes.c_float, vp]
        L.tgo_surrogate_adam_step.restype = i32
        L.tgo_surrogate_get_moments.argtypes = [vp, vp, vp, ctypes.POINTER(ctypes.c_int64), vp]
        L.tgo_surrogate_get_moments.restype = i32
        L.tgo_surrogate_get_batch.argtypes = [vp, i32, i64, vp, vp]
        L.tgo_surrogate_get_batch.restype = i32
        for f in (L.tgo_surrogate_create, L.tgo_surrogate_param_count, L.tgo_surrogate_init,
                  L.tgo_surrogate_set_params, L.tgo_surrogate_get_params, L.tgo_surrogate_pairs,
                  L.tgo_surrogate_score, L.tgo_surrogate_grad, L.tgo_surrogate_train_step,
                  L.tgo_surrogate_search, L.tgo_random_search):
            f.restype = i32
        L.tgo_server_config_default.argtypes = [vp]
        L.tgo_server_config_default.restype = None
        L.tgo_server_create.argtypes = [M, vp, vp, ctypes.POINTER(vp)]
        L.tgo_server_submit.argtypes = [vp, vp, i32, ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint64)]
        L.tgo_server_poll.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_int)]
        L.tgo_server_drain.argtypes = [vp, i64]
        L.tgo_server_get_stats.argtypes = [vp, vp]
        L.tgo_server_replay.argtypes = [vp, vp, vp, vp, i32, vp, i64]
        L.tgo_server_destroy.argtypes = [vp]
        L.tgo_server_destroy.restype = None
        for f in (L.tgo_server_create, L.tgo_server_submit, L.tgo_server_poll, L.tgo_server_drain,
                  L.tgo_server_get_stats, L.tgo_server_replay):
            f.restype = i32
        L.tgo_hw_create.argtypes = [i32, i64, i64, ctypes.POINTER(vp)]
        L.tgo_hw_destroy.argtypes = [vp]
        L.tgo_hw_destroy.restype = None
        L.tgo_hw_run.argtypes = [vp, vp, i32, vp, i32, ctypes.POINTER(ctypes.c_int64), vp]
        L.tgo_hw_overlap.argtypes = [vp, i64, i64, i64, vp]
        L.tgo_hw_run_rounds.argtypes = [vp, vp, i32, i32, vp, i32, ctypes.POINTER(ctypes.c_int64), vp]
        L.tgo_hw_run_rounds.restype = i32
        L.tgo_hw_run_mem.argtypes = [vp, vp, i32, vp, vp, i64, i32, ctypes.POINTER(ctypes.c_int64), vp]
        L.tgo_hw_run_mem.restype = i32
        L.tgo_hw_run_proxy.argtypes = [vp, M, vp, vp, i32, i32, ctypes.POINTER(ctypes.c_int64), vp, vp, vp]
        L.tgo_hw_run_proxy.restype = i32
        L.tgo_fit_line.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.tgo_fit_overlap.argtypes = [vp, vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        for f in (L.tgo_hw_create, L.tgo_hw_run, L.tgo_hw_overlap, L.tgo_fit_line, L.tgo_fit_overlap):
            f.restype = i32
        L.tgo_plan_destroy.argtypes = [vp]
        L.tgo_plan_destroy.restype = None
        for f in (L.tgo_evaluate, L.tgo_exhaustive, L.tgo_heuristic, L.tgo_rounds, L.tgo_rank, L.tgo_unrank,
                  L.tgo_plan_create, L.tgo_plan_autotune, L.tgo_plan_describe, L.tgo_batch):
            f.restype = i32
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != TGO_OK:
        L = lib()
        raise TgoError(rc, where, f"{L.tgo_strerror(rc).decode()}: {L.tgo_last_error().decode()}")


def _stream(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _dev_tensor(x, dtype, shape_last=None, name="tensor"):
    import torch
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {x.dtype}")
    if not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape_last is not None and (x.dim() < 1 or x.shape[-1] != shape_last):
        raise ValueError(f"{name} must have last dimension {shape_last}")
    return x


def evaluate(tasks, orders, model: Model = DEFAULT, out=None, stream=None):
    """T (int64 ns) for each row of ``orders`` (uint8 [m, n]); tasks int64 [n, 3]."""
    import torch
    _dev_tensor(tasks, torch.int64, 3, "tasks")
    _dev_tensor(orders, torch.uint8, None, "orders")
    n = tasks.shape[0]
    if orders.dim() != 2 or orders.shape[1] != n:
        raise ValueError("orders must be [m, n]")
    m = orders.shape[0]
    if out is None:
        out = torch.empty(m, dtype=torch.int64, device=tasks.device)
    _dev_tensor(out, torch.int64, None, "out")
    _check(lib().tgo_evaluate(ctypes.byref(model._c()), tasks.data_ptr(), n, orders.data_ptr(), m,
                              out.data_ptr(), _stream(stream)), "tgo_evaluate")
    return out


def exhaustive(tasks, model: Model = DEFAULT, per_order: bool = False, summary=None, stream=None):
    """Enumerate all n! orderings.  Returns (summary uint8[112] device tensor,
    per-ordering int64[n!] device tensor or None)."""
    import math
    import torch
    _dev_tensor(tasks, torch.int64, 3, "tasks")
    n = tasks.shape[0]
    po = None
    if per_order:
        po = torch.empty(math.factorial(n), dtype=torch.int64, device=tasks.device)
    if summary is None:
        summary = torch.empty(SUMMARY_DTYPE.itemsize, dtype=torch.uint8, device=tasks.device)
    _check(lib().tgo_exhaustive(ctypes.byref(model._c()), tasks.data_ptr(), n,
                                po.data_ptr() if po is not None else None, summary.data_ptr(),
                                _stream(stream)), "tgo_exhaustive")
    return summary, po


def exhaustive_noalloc(tasks, summary, per_order=None, model: Model = DEFAULT, stream=None):
    """tgo_exhaustive_noalloc: the same enumeration with the library's fixed
    per-device scratch (the call allocates nothing; the caller passes the
    summary, uint8[136], and optionally the per-ordering int64[n!] buffer).
    Calls that overlap on one device race on that scratch."""
    import math
    import torch
    _dev_tensor(tasks, torch.int64, 3, "tasks")
    _dev_tensor(summary, torch.uint8, None, "summary")
    if summary.numel() < SUMMARY_DTYPE.itemsize:
        raise ValueError("summary must hold 136 bytes")
    n = tasks.shape[0]
    if per_order is not None:
        _dev_tensor(per_order, torch.int64, None, "per_order")
        if per_order.numel() < math.factorial(n):
            raise ValueError("per_order must hold n! entries")
    _check(lib().tgo_exhaustive_noalloc(ctypes.byref(model._c()), tasks.data_ptr(), n,
                                        per_order.data_ptr() if per_order is not None else None,
                                        summary.data_ptr(), _stream(stream)), "tgo_exhaustive_noalloc")
    return summary, per_order


def exhaustive_cke(tasks, units, capacity: int, model: Model = DEFAULT, per_order: bool = False, summary=None,
                   stream=None):
    """Every ordering with concurrent kernels: task x's kernel holds units[x]
    (int32 [n] device tensor) of ``capacity`` while it runs.  Returns (summary
    uint8[136] device tensor with Algorithm 1 under the same rule in heur /
    heur_ns, per-ordering int64 device tensor or None)."""
    import math
    import torch
    _dev_tensor(tasks, torch.int64, 3, "tasks")
    _dev_tensor(units, torch.int32, None, "units")
    n = tasks.shape[0]
    if units.numel() != n:
        raise ValueError("one unit count per task")
    po = torch.empty(math.factorial(n), dtype=torch.int64, device=tasks.device) if per_order else None
    if summary is None:
        summary = torch.empty(SUMMARY_DTYPE.itemsize, dtype=torch.uint8, device=tasks.device)
    _check(lib().tgo_exhaustive_cke(ctypes.byref(model._c()), tasks.data_ptr(), units.data_ptr(), n, capacity,
                                    po.data_ptr() if po is not None else None, summary.data_ptr(),
                                    _stream(stream)), "tgo_exhaustive_cke")
    return summary, po


def evaluate_cke(tasks, units, capacity: int, orders, model: Model = DEFAULT, out=None, stream=None):
    """T (int64) of each row of ``orders`` (uint8 [m, n]) with concurrent kernels."""
    import torch
    _dev_tensor(tasks, torch.int64, 3, "tasks")
    _dev_tensor(units, torch.int32, None, "units")
    _dev_tensor(orders, torch.uint8, None, "orders")
    n = tasks.shape[0]
    if orders.dim() != 2 or orders.shape[1] != n or units.numel() != n:
        raise ValueError("orders must be [m, n] and units [n]")
    m = orders.shape[0]
    if out is None:
        out = torch.empty(m, dtype=torch.int64, device=tasks.device)
    _check(lib().tgo_evaluate_cke(ctypes.byref(model._c()), tasks.data_ptr(), units.data_ptr(), n, capacity,
                                  orders.data_ptr(), m, out.data_ptr(), _stream(stream)), "tgo_evaluate_cke")
    return out


def predict(tasks, order, model: Model = DEFAULT) -> int:
    """T (ns) of one ordering of host tasks (int64 [n, 3]), computed on the device."""
    t = np.ascontiguousarray(np.asarray(tasks, dtype=np.int64).reshape(-1, 3))
    o = np.ascontiguousarray(np.asarray(order, dtype=np.uint8))
    out = ctypes.c_int64()
    _check(lib().tgo_predict(ctypes.byref(model._c()), t.ctypes.data, len(t), o.ctypes.data, ctypes.byref(out)),
           "tgo_predict")
    return int(out.value)


def rounds(tasks, workers: int, rounds: int, model: Model = DEFAULT, per_order: bool = False,
           summary=None, stream=None):
    """Several workers offloading dependent tasks: task (w, r) at row
    w * rounds + r of ``tasks`` (int64 [workers * rounds, 3]).  Returns
    (summary uint8[136] device tensor -- NoReorder over all (workers!)^rounds
    orderings, plus the Heuristic setup in heur / heur_ns --, per-ordering
    int64 device tensor or None, uint16 group-end mask device tensor)."""
    import math
    import torch
    _dev_tensor(tasks, torch.int64, 3, "tasks")
    if tasks.shape[0] != workers * rounds:
        raise ValueError("tasks must have workers * rounds rows")
    po = None
    if per_order:
        po = torch.empty(math.factorial(workers) ** rounds, dtype=torch.int64, device=tasks.device)
    if summary is None:
        summary = torch.empty(SUMMARY_DTYPE.itemsize, dtype=torch.uint8, device=tasks.device)
    groups = torch.zeros(1, dtype=torch.int16, device=tasks.device)
    _check(lib().tgo_rounds(ctypes.byref(model._c()), tasks.data_ptr(), workers, rounds,
                            po.data_ptr() if po is not None else None, summary.data_ptr(),
                            groups.data_ptr(), _stream(stream)), "tgo_rounds")
    return summary, po, groups


def exhaustive_mem(tasks, mem, capacity: int, model: Model = DEFAULT, per_order: bool = False, summary=None,
                   stream=None):
    """Every ordering under a device-memory limit: task x holds mem[x] bytes
    (int64 [n] device tensor) from its HtD start to its DtH end, at most
    ``capacity`` at once.  Returns (summary uint8 device tensor with the
    heuristic under the limit in heur / heur_ns, per-ordering int64 device
    tensor or None)."""
    import math
    import torch
    _dev_tensor(tasks, torch.int64, 3, "tasks")
    _dev_tensor(mem, torch.int64, None, "mem")
    n = tasks.shape[0]
    if mem.shape != (n,):
        raise ValueError("mem must be int64 [n]")
    po = torch.empty(math.factorial(n), dtype=torch.int64, device=tasks.device) if per_order else None
    if summary is None:
        summary = torch.empty(SUMMARY_DTYPE.itemsize, dtype=torch.uint8, device=tasks.device)
    _check(lib().tgo_exhaustive_mem(ctypes.byref(model._c()), tasks.data_ptr(), mem.data_ptr(), n, int(capacity),
                                    po.data_ptr() if po is not None else None, summary.data_ptr(),
                                    _stream(stream)), "tgo_exhaustive_mem")
    return summary, po


def evaluate_mem(tasks, mem, capacity: int, orders, model: Model = DEFAULT, out=None, stream=None):
    """T (int64 ns) of each row of ``orders`` (uint8 [m, n]) under the
    device-memory limit of ``exhaustive_mem``."""
    import torch
    _dev_tensor(tasks, torch.int64, 3, "tasks")
    _dev_tensor(mem, torch.int64, None, "mem")
    _dev_tensor(orders, torch.uint8, None, "orders")
    n = tasks.shape[0]
    if mem.shape != (n,):
        raise ValueError("mem must be int64 [n]")
    if orders.dim() != 2 or orders.shape[1] != n:
        raise ValueError("orders must be [m, n]")
    m = orders.shape[0]
    if out is None:
        out = torch.empty(m, dtype=torch.int64, device=tasks.device)
    _dev_tensor(out, torch.int64, None, "out")
    _check(lib().tgo_evaluate_mem(ctypes.byref(model._c()), tasks.data_ptr(), mem.data_ptr(), n, int(capacity),
                                  orders.data_ptr(), m, out.data_ptr(), _stream(stream)), "tgo_evaluate_mem")
    return out


def valu_probe(blocks: int, iters: int, stream=None):
    """Launch the integer issue probe of the calibration library
    (libtgo_probe.so, tgo_probe_valu): a measurement of the device for the
    ALU roofline, not part of the model."""
    import torch
    path = os.path.join(_PKG, "libtgo_probe.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run python -m paper_1806_10113_amd.build")
    P = ctypes.CDLL(path)
    P.tgo_probe_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    P.tgo_probe_valu.restype = ctypes.c_int
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    rc = P.tgo_probe_valu(int(blocks), int(iters), sink.data_ptr(), _stream(stream))
    if rc != 0:
        raise TgoError(rc, "tgo_probe_valu", "bad argument" if rc == -1 else "launch error")
    return sink


def read_groups(groups) -> list:
    """Positions that end a proxy task group, from the uint16 mask."""
    m = int(groups.cpu().numpy().view("<u2")[0])
    return [j for j in range(16) if (m >> j) & 1]


def read_summary(summary) -> dict:
    """Copy a device summary to the host and decode it."""
    raw = summary.cpu().numpy().view(SUMMARY_DTYPE)[0]
    return _decode(raw)


def _decode(raw) -> dict:
    n = int(raw["n"])
    d = {k: raw[k].item() for k in SUMMARY_DTYPE.names if k not in ("best", "worst", "heur")}
    d["sum"] = int(raw["sum_lo"]) | (int(raw["sum_hi"]) << 64)
    d["best"] = [int(v) for v in raw["best"][:n]]
    d["worst"] = [int(v) for v in raw["worst"][:n]]
    d["heur"] = [int(v) for v in raw["heur"][:n]]
    return d


def read_summaries(summaries) -> list:
    """Decode a device array of summaries (uint8 [G, 136])."""
    raw = summaries.cpu().numpy().reshape(-1).view(SUMMARY_DTYPE)
    return [_decode(r) for r in raw]


def heuristic(tasks, offs, model: Model = DEFAULT, stream=None):
    """Algorithm 1 on every group of a CSR batch.  Returns (orders uint8 [G, 16], T int64 [G])."""
    import torch
    _dev_tensor(tasks, torch.int64, 3, "tasks")
    _dev_tensor(offs, torch.int32, None, "offs")
    g = offs.shape[0] - 1
    orders = torch.empty((max(g, 0), 16), dtype=torch.uint8, device=tasks.device)
    ns = torch.empty(max(g, 0), dtype=torch.int64, device=tasks.device)
    _check(lib().tgo_heuristic(ctypes.byref(model._c()), tasks.data_ptr(), offs.data_ptr(), g,
                               orders.data_ptr(), ns.data_ptr(), _stream(stream)), "tgo_heuristic")
    return orders, ns


class Plan:
    """Batched enumeration plan (device workspace, captured graph, tuned decomposition)."""

    def __init__(self, model: Model = DEFAULT, max_groups: int = 4096, max_n: int = 12, mem_budget: int = 0):
        self._h = ctypes.c_void_p()
        self.model = model
        self.max_groups = max_groups
        _check(lib().tgo_plan_create(ctypes.byref(model._c()), max_groups, max_n, mem_budget,
                                     ctypes.byref(self._h)), "tgo_plan_create")

    def close(self):
        if self._h:
            lib().tgo_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _out(self, offs, out):
        import torch
        g = offs.shape[0] - 1
        if out is None:
            out = torch.empty((g, SUMMARY_DTYPE.itemsize), dtype=torch.uint8, device=offs.device)
        return g, out

    def autotune(self, tasks, offs, out=None, stream=None):
        import torch
        _dev_tensor(tasks, torch.int64, 3, "tasks")
        _dev_tensor(offs, torch.int32, None, "offs")
        g, out = self._out(offs, out)
        _check(lib().tgo_plan_autotune(self._h, tasks.data_ptr(), offs.data_ptr(), g, out.data_ptr(),
                                       _stream(stream)), "tgo_plan_autotune")
        return self.describe()

    def describe(self) -> dict:
        import json
        buf = ctypes.create_string_buffer(1024)
        _check(lib().tgo_plan_describe(self._h, buf, 1024), "tgo_plan_describe")
        return json.loads(buf.value.decode())

    def set_decomposition(self, desc: dict):
        """Restore a decomposition that describe() reported (m_by_n, lane_mult,
        blocks), e.g. saved from a tuning run, instead of tuning again."""
        m = np.ascontiguousarray(np.asarray(desc["m_by_n"], dtype=np.int32))
        if m.shape != (12,):
            raise ValueError("m_by_n must hold 12 entries (group sizes 1..12)")
        _check(lib().tgo_plan_set_decomposition(self._h, m.ctypes.data, int(desc["lane_mult"]),
                                                int(desc["blocks"])), "tgo_plan_set_decomposition")

    def run(self, tasks, offs, out=None, stream=None):
        """Summaries (uint8 [G, 136] device tensor) for every group of the batch."""
        import torch
        _dev_tensor(tasks, torch.int64, 3, "tasks")
        _dev_tensor(offs, torch.int32, None, "offs")
        g, out = self._out(offs, out)
        _dev_tensor(out, torch.uint8, SUMMARY_DTYPE.itemsize, "out")
        _check(lib().tgo_batch(self._h, tasks.data_ptr(), offs.data_ptr(), g, out.data_ptr(),
                               _stream(stream)), "tgo_batch")
        return out


SEARCH_DTYPE = np.dtype([
    ("best_ns", "<i8"), ("heur_ns", "<i8"), ("cand_best_ns", "<i8"), ("best_sample", "<u8"),
    ("status", "<i4"), ("n", "<i4"), ("from_heuristic", "<i4"), ("pad", "<i4"), ("best", "u1", (16,)),
])
assert SEARCH_DTYPE.itemsize == 64
SURROGATE_PARAMS = 144385


def read_search(results) -> list:
    raw = results.cpu().numpy().reshape(-1).view(SEARCH_DTYPE)
    out = []
    for r in raw:
        n = int(r["n"])
        d = {k: r[k].item() for k in SEARCH_DTYPE.names if k not in ("best", "pad")}
        d["best"] = [int(v) for v in r["best"][:n]]
        out.append(d)
    return out


def _groups(tasks, offs):
    import torch
    _dev_tensor(tasks, torch.int64, 3, "tasks")
    _dev_tensor(offs, torch.int32, None, "offs")
    return offs.shape[0] - 1


def pairs(tasks, offs, per_group: int, seed: int, model: Model = DEFAULT, stream=None):
    """Exact training pairs: (orders uint8 [P,16], gid int32 [P], T int64 [P], status int32 [G])."""
    import torch
    g = _groups(tasks, offs)
    P = g * per_group
    dev = tasks.device
    orders = torch.empty((P, 16), dtype=torch.uint8, device=dev)
    gid = torch.empty(P, dtype=torch.int32, device=dev)
    T = torch.empty(P, dtype=torch.int64, device=dev)
    status = torch.empty(g, dtype=torch.int32, device=dev)
    _check(lib().tgo_surrogate_pairs(ctypes.byref(model._c()), tasks.data_ptr(), offs.data_ptr(), g,
                                     per_group, seed, status.data_ptr(), orders.data_ptr(),
                                     gid.data_ptr(), T.data_ptr(), _stream(stream)),
           "tgo_surrogate_pairs")
    return orders, gid, T, status


def random_search(tasks, offs, samples: int, seed: int, model: Model = DEFAULT, stream=None):
    """Plain exact search (heuristic + sampled orderings scored exactly); uint8 [G, 64] results."""
    import torch
    g = _groups(tasks, offs)
    out = torch.empty((g, SEARCH_DTYPE.itemsize), dtype=torch.uint8, device=tasks.device)
    _check(lib().tgo_random_search(ctypes.byref(model._c()), tasks.data_ptr(), offs.data_ptr(), g,
                                   samples, seed, out.data_ptr(), _stream(stream)), "tgo_random_search")
    return out


class Surrogate:
    """The learned proposal: bf16 MLP on the matrix cores, float32 masters, Adam."""

    def __init__(self, max_rows: int = 1 << 18, max_groups: int = 4096):
        self._h = ctypes.c_void_p()
        self.max_rows = max_rows
        _check(lib().tgo_surrogate_create(max_rows, max_groups, ctypes.byref(self._h)),
               "tgo_surrogate_create")

    def close(self):
        if self._h:
            lib().tgo_surrogate_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, seed: int, stream=None):
        _check(lib().tgo_surrogate_init(self._h, seed, _stream(stream)), "tgo_surrogate_init")

    def save(self, path: str):
        _check(lib().tgo_surrogate_save(self._h, os.fsencode(path)), "tgo_surrogate_save")

    def load(self, path: str):
        _check(lib().tgo_surrogate_load(self._h, os.fsencode(path)), "tgo_surrogate_load")

    def set_params(self, params: np.ndarray, stream=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.size == SURROGATE_PARAMS
        _check(lib().tgo_surrogate_set_params(self._h, p.ctypes.data, _stream(stream)),
               "tgo_surrogate_set_params")

    def get_params(self, stream=None) -> np.ndarray:
        p = np.empty(SURROGATE_PARAMS, dtype=np.float32)
        _check(lib().tgo_surrogate_get_params(self._h, p.ctypes.data, _stream(stream)),
               "tgo_surrogate_get_params")
        return p

    def score(self, tasks, offs, orders, gid, stream=None):
        import torch
        g = _groups(tasks, offs)
        rows = orders.shape[0]
        out = torch.empty(rows, dtype=torch.float32, device=tasks.device)
        _check(lib().tgo_surrogate_score(self._h, tasks.data_ptr(), offs.data_ptr(), g,
                                         orders.data_ptr(), gid.data_ptr(), rows, out.data_ptr(),
                                         _stream(stream)), "tgo_surrogate_score")
        return out

    def grad(self, tasks, offs, orders, gid, T, stream=None):
        import torch
        g = _groups(tasks, offs)
        rows = orders.shape[0]
        grad = torch.empty(SURROGATE_PARAMS, dtype=torch.float32, device=tasks.device)
        loss = torch.empty(1, dtype=torch.float32, device=tasks.device)
        _check(lib().tgo_surrogate_grad(self._h, tasks.data_ptr(), offs.data_ptr(), g, orders.data_ptr(),
                                        gid.data_ptr(), T.data_ptr(), rows, grad.data_ptr(),
                                        loss.data_ptr(), _stream(stream)), "tgo_surrogate_grad")
        return grad, loss

    def train_step(self, tasks, offs, orders, gid, T, lr: float, loss=None, stream=None):
        import torch
        g = _groups(tasks, offs)
        rows = orders.shape[0]
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=tasks.device)
        _check(lib().tgo_surrogate_train_step(self._h, tasks.data_ptr(), offs.data_ptr(), g,
                                              orders.data_ptr(), gid.data_ptr(), T.data_ptr(), rows,
                                              lr, loss.data_ptr(), _stream(stream)),
               "tgo_surrogate_train_step")
        return loss

    def adam_step(self, grad, lr: float, stream=None):
        """One Adam step of the masters with a given float32 device gradient."""
        import torch
        _dev_tensor(grad, torch.float32, None, "grad")
        if grad.numel() != SURROGATE_PARAMS:
            raise ValueError("grad must hold every parameter")
        _check(lib().tgo_surrogate_adam_step(self._h, grad.data_ptr(), lr, _stream(stream)),
               "tgo_surrogate_adam_step")

    def moments(self):
        """(m, v, step): Adam's moments as float32 host arrays and the step count."""
        m = np.empty(SURROGATE_PARAMS, dtype=np.float32)
        v = np.empty(SURROGATE_PARAMS, dtype=np.float32)
        t = ctypes.c_int64()
        _check(lib().tgo_surrogate_get_moments(self._h, m.ctypes.data, v.ctypes.data, ctypes.byref(t), None),
               "tgo_surrogate_get_moments")
        return m, v, t.value

    BATCH_FEATURES, BATCH_H1, BATCH_H2, BATCH_H3, BATCH_SCORE, BATCH_G3, BATCH_G2, BATCH_G1 = range(8)

    def batch_values(self, what: int, rows: int) -> np.ndarray:
        """A stored value of the last grad() batch, row-major: bf16 values as
        float64 (features [rows, 48], h1..h3 and the gradients G3, G2, G1
        [rows, 256]) or the float32 scores [rows]."""
        if what == self.BATCH_SCORE:
            out = np.empty(rows, dtype=np.float32)
        else:
            out = np.empty((rows, 48 if what == self.BATCH_FEATURES else 256), dtype=np.uint16)
        _check(lib().tgo_surrogate_get_batch(self._h, what, rows, out.ctypes.data, None),
               "tgo_surrogate_get_batch")
        if what == self.BATCH_SCORE:
            return out
        return (out.astype(np.uint32) << 16).view(np.float32).astype(np.float64)

    def search(self, tasks, offs, samples: int, topk: int, seed: int, model: Model = DEFAULT,
               keys=None, stream=None):
        import torch
        g = _groups(tasks, offs)
        if keys is not None:
            _dev_tensor(keys, torch.int32, None, "keys")
        out = torch.empty((g, SEARCH_DTYPE.itemsize), dtype=torch.uint8, device=tasks.device)
        _check(lib().tgo_surrogate_search(self._h, ctypes.byref(model._c()), tasks.data_ptr(),
                                          offs.data_ptr(), keys.data_ptr() if keys is not None else None,
                                          g, samples, topk, seed, out.data_ptr(), _stream(stream)),
               "tgo_surrogate_search")
        return out

    def candidates(self, tasks, offs, samples: int, topk: int, seed: int, model: Model = DEFAULT,
                   keys=None, stream=None):
        """The search's candidate keys: uint64 [groups, topk] device tensor
        (score order bits << 32 | sample index, ascending; ~0 = none)."""
        import torch
        g = _groups(tasks, offs)
        if keys is not None:
            _dev_tensor(keys, torch.int32, None, "keys")
        out = torch.empty((g, topk), dtype=torch.int64, device=tasks.device)
        _check(lib().tgo_surrogate_candidates(self._h, ctypes.byref(model._c()), tasks.data_ptr(),
                                              offs.data_ptr(), keys.data_ptr() if keys is not None else None,
                                              g, samples, topk, seed, out.data_ptr(), _stream(stream)),
               "tgo_surrogate_candidates")
        return out


class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("streams", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("max_batch_large", ctypes.c_int32),
                ("small_max_n", ctypes.c_int32), ("topk", ctypes.c_int32), ("window_us", ctypes.c_int32),
                ("samples", ctypes.c_int64), ("seed", ctypes.c_uint64)]


SERVER_RESULT_DTYPE = np.dtype([
    ("id", "<u8"), ("t_arrive_ns", "<i8"), ("t_admit_ns", "<i8"), ("t_done_ns", "<i8"),
    ("n", "<i4"), ("path", "<i4"), ("status", "<i4"), ("pad", "<i4"), ("best_ns", "<i8"),
    ("heur_ns", "<i8"), ("best", "u1", (16,)),
])
assert SERVER_RESULT_DTYPE.itemsize == 80


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("rejected", ctypes.c_uint64),
                ("in_use_bytes", ctypes.c_int64), ("max_in_use_bytes", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("max_queued", ctypes.c_int64),
                ("base_bytes", ctypes.c_int64), ("ring_rows", ctypes.c_int64 * 2),
                ("budget_bytes", ctypes.c_int64)]


def server_config(**kw) -> ServerConfig:
    c = ServerConfig()
    lib().tgo_server_config_default(ctypes.byref(c))
    for k, v in kw.items():
        setattr(c, k, v)
    return c


class Server:
    """Continuous-batching request loop (host scheduler thread, HIP streams)."""

    def __init__(self, model: Model = DEFAULT, config: ServerConfig | None = None,
                 surrogate: "Surrogate | None" = None):
        self._h = ctypes.c_void_p()
        self.config = config or server_config()
        _check(lib().tgo_server_create(ctypes.byref(model._c()), ctypes.byref(self.config),
                                       surrogate._h if surrogate is not None else None,
                                       ctypes.byref(self._h)), "tgo_server_create")

    def close(self):
        if self._h:
            lib().tgo_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, tasks, key: int = 0) -> int:
        t = np.ascontiguousarray(np.asarray(tasks, dtype=np.int64).reshape(-1, 3))
        rid = ctypes.c_uint64()
        _check(lib().tgo_server_submit(self._h, t.ctypes.data, len(t), key, ctypes.byref(rid)),
               "tgo_server_submit")
        return rid.value

    def poll(self, max_results: int = 4096, raise_on_error: bool = True):
        """Finished results.  After a device error the C call still hands back
        what finished (failed requests carry status TGO_EDEVICE) and returns
        TGO_EDEVICE: with raise_on_error=False this returns (results, code)."""
        out = np.zeros(max_results, dtype=SERVER_RESULT_DTYPE)
        k = ctypes.c_int()
        rc = lib().tgo_server_poll(self._h, out.ctypes.data, max_results, ctypes.byref(k))
        if not raise_on_error:
            return out[:k.value], rc
        _check(rc, "tgo_server_poll")
        return out[:k.value]

    def drain(self, timeout_ms: int = 60_000):
        _check(lib().tgo_server_drain(self._h, timeout_ms), "tgo_server_drain")

    def stats(self) -> dict:
        s = ServerStats()
        _check(lib().tgo_server_get_stats(self._h, ctypes.byref(s)), "tgo_server_get_stats")
        d = {k: getattr(s, k) for k, _ in ServerStats._fields_}
        d["ring_rows"] = list(d["ring_rows"])
        return d

    def replay(self, tasks, offs, arrival_ns, timeout_ms: int = 600_000) -> np.ndarray:
        t = np.ascontiguousarray(np.asarray(tasks, dtype=np.int64).reshape(-1, 3))
        o = np.ascontiguousarray(np.asarray(offs, dtype=np.int32))
        a = np.ascontiguousarray(np.asarray(arrival_ns, dtype=np.int64))
        n = len(o) - 1
        out = np.zeros(n, dtype=SERVER_RESULT_DTYPE)
        _check(lib().tgo_server_replay(self._h, t.ctypes.data, o.ctypes.data, a.ctypes.data, n,
                                       out.ctypes.data, timeout_ms), "tgo_server_replay")
        return out


HW_TASK_DTYPE = np.dtype([("htd_bytes", "<i8"), ("dth_bytes", "<i8"), ("kern_elems", "<i8"),
                          ("kern_iters", "<i4"), ("kern_kind", "<i4")])
HW_KERNEL_HBM, HW_KERNEL_ALU = 0, 1
HW_TIMES_DTYPE = np.dtype([("start_ns", "<i8", (3,)), ("end_ns", "<i8", (3,))])


class HwRunner:
    """Real HtD / kernel / DtH tasks on the current device (tgo_hw_*)."""

    def __init__(self, max_tasks: int, max_bytes: int, max_kern_elems: int):
        self._h = ctypes.c_void_p()
        _check(lib().tgo_hw_create(max_tasks, max_bytes, max_kern_elems, ctypes.byref(self._h)),
               "tgo_hw_create")

    def close(self):
        if self._h:
            lib().tgo_hw_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, tasks: np.ndarray, order, dma_engines: int = 2):
        """tasks: HW_TASK_DTYPE [n].  Returns (makespan ns, HW_TIMES_DTYPE [n])."""
        tasks = np.ascontiguousarray(tasks, dtype=HW_TASK_DTYPE)
        n = len(tasks)
        o = np.ascontiguousarray(order, dtype=np.uint8)
        times = np.zeros(n, dtype=HW_TIMES_DTYPE)
        total = ctypes.c_int64()
        _check(lib().tgo_hw_run(self._h, tasks.ctypes.data, n, o.ctypes.data, dma_engines,
                                ctypes.byref(total), times.ctypes.data), "tgo_hw_run")
        return int(total.value), times

    def run_rounds(self, tasks: np.ndarray, workers: int, rounds: int, seq, dma_engines: int = 2):
        """Dependent tasks (task (w, r) at row w * rounds + r), launched in
        ``seq`` round by round.  Returns (makespan ns, HW_TIMES_DTYPE [n])."""
        tasks = np.ascontiguousarray(tasks, dtype=HW_TASK_DTYPE)
        o = np.ascontiguousarray(seq, dtype=np.uint8)
        times = np.zeros(len(tasks), dtype=HW_TIMES_DTYPE)
        total = ctypes.c_int64()
        _check(lib().tgo_hw_run_rounds(self._h, tasks.ctypes.data, workers, rounds, o.ctypes.data, dma_engines,
                                       ctypes.byref(total), times.ctypes.data), "tgo_hw_run_rounds")
        return int(total.value), times

    def run_mem(self, tasks: np.ndarray, order, mem, capacity: int, dma_engines: int = 2):
        """``run`` under a device-memory limit (tgo_hw_run_mem): mem[x] bytes
        per task, at most ``capacity`` held.  Returns (makespan ns,
        HW_TIMES_DTYPE [n])."""
        tasks = np.ascontiguousarray(tasks, dtype=HW_TASK_DTYPE)
        o = np.ascontiguousarray(order, dtype=np.uint8)
        m = np.ascontiguousarray(np.asarray(mem, dtype=np.int64))
        times = np.zeros(len(tasks), dtype=HW_TIMES_DTYPE)
        total = ctypes.c_int64()
        _check(lib().tgo_hw_run_mem(self._h, tasks.ctypes.data, len(tasks), o.ctypes.data, m.ctypes.data,
                                    int(capacity), dma_engines, ctypes.byref(total), times.ctypes.data),
               "tgo_hw_run_mem")
        return int(total.value), times

    def run_proxy(self, tasks: np.ndarray, durations, workers: int, rounds: int, model: Model = DEFAULT):
        """The Heuristic setup with a host proxy (tgo_hw_run_proxy).  Returns
        (makespan ns, submission order, group-end positions, HW_TIMES_DTYPE [n])."""
        tasks = np.ascontiguousarray(tasks, dtype=HW_TASK_DTYPE)
        dur = np.ascontiguousarray(np.asarray(durations, dtype=np.int64).reshape(-1, 3))
        n = len(tasks)
        seq = np.zeros(16, dtype=np.uint8)
        groups = np.zeros(1, dtype=np.uint16)
        times = np.zeros(n, dtype=HW_TIMES_DTYPE)
        total = ctypes.c_int64()
        _check(lib().tgo_hw_run_proxy(self._h, ctypes.byref(model._c()), tasks.ctypes.data, dur.ctypes.data,
                                      workers, rounds, ctypes.byref(total), seq.ctypes.data, groups.ctypes.data,
                                      times.ctypes.data), "tgo_hw_run_proxy")
        ends = [j for j in range(16) if (int(groups[0]) >> j) & 1]
        return int(total.value), [int(v) for v in seq[:n]], ends, times

    def overlap(self, htd_bytes: int, dth_bytes: int, delay_ns: int) -> np.ndarray:
        out = np.zeros(4, dtype=np.int64)
        _check(lib().tgo_hw_overlap(self._h, htd_bytes, dth_bytes, delay_ns, out.ctypes.data),
               "tgo_hw_overlap")
        return out


def fit_line(x, y):
    """(slope, intercept) of the least-squares line (tgo_fit_line)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(lib().tgo_fit_line(x.ctypes.data, y.ctypes.data, len(x), ctypes.byref(a), ctypes.byref(b)),
           "tgo_fit_line")
    return a.value, b.value


def fit_overlap(times, solo):
    """(rho_htd, rho_dth) from overlap experiments (tgo_fit_overlap)."""
    t = np.ascontiguousarray(times, dtype=np.int64).reshape(-1, 4)
    so = np.ascontiguousarray(solo, dtype=np.int64).reshape(-1, 2)
    a, b = ctypes.c_double(), ctypes.c_double()
    _check(lib().tgo_fit_overlap(t.ctypes.data, so.ctypes.data, len(t), ctypes.byref(a), ctypes.byref(b)),
           "tgo_fit_overlap")
    return a.value, b.value


def rank(order) -> int:
    o = np.ascontiguousarray(np.asarray(order, dtype=np.uint8))
    r = ctypes.c_uint64()
    _check(lib().tgo_rank(len(o), o.ctypes.data, ctypes.byref(r)), "tgo_rank")
    return r.value


def unrank(n: int, r: int):
    o = np.zeros(16, dtype=np.uint8)
    _check(lib().tgo_unrank(n, r, o.ctypes.data), "tgo_unrank")
    return [int(v) for v in o[:n]]
