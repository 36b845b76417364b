"""Python binding of libtnc's C ABI (include/tnc.h): the same function names, argument
marshalling only.  Pointers are passed as ints (for example torch's data_ptr()); every
contraction step runs inside the library.

The library is loaded from this package directory; a missing build raises instead of
falling back to anything else.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtnc.so")

TNC_OK = 0
TNC_E_INVALID = -1
TNC_E_OOM = -2
TNC_E_HIP = -3
TNC_E_UNSUPPORTED = -4
TNC_E_BUSY = -5
TNC_E_NOT_FOUND = -6
TNC_E_INTERNAL = -7

TNC_C64, TNC_FP16X3, TNC_BF16X3, TNC_FP16X3_3M, TNC_BF16X3_3M = range(5)

KIND_NAMES = ("permute", "gemm", "stream", "slice_leaves", "slice_sum", "splitk_reduce",
              "scale_records")

EXPORTS = (
    "tnc_last_error", "tnc_net_create", "tnc_net_set_path", "tnc_net_set_slices",
    "tnc_net_set_slices_wide", "tnc_net_set_targets", "tnc_plan_create", "tnc_plan_workspace_bytes", "tnc_plan_stats", "tnc_plan_work",
    "tnc_contract", "tnc_contract_range", "tnc_sample", "tnc_sample_metropolis",
    "tnc_sample_frugal", "tnc_sample_noalloc", "tnc_plan_destroy", "tnc_net_destroy",
    "tnc_plan_autotune", "tnc_plan_batch_slices", "tnc_plan_n_launches", "tnc_plan_launch_info", "tnc_plan_set_timing", "tnc_plan_timing",
    "tnc_plan_launch_timing",
    "tnc_server_create", "tnc_server_submit", "tnc_server_poll", "tnc_server_pending",
    "tnc_server_destroy",
)


class TncError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tnc error {code}: {msg}")
        self.code = code


class _Desc(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_tensors", ctypes.c_int32),
                ("ranks", ctypes.c_void_p), ("labels", ctypes.c_void_p),
                ("data", ctypes.c_void_p), ("out_label", ctypes.c_void_p)]


class StepInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("invariant", ctypes.c_int32),
                ("rows", ctypes.c_int64), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("k", ctypes.c_int64), ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
                ("config", ctypes.c_int32), ("k_splits", ctypes.c_int32),
                ("row_mode", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("n_amplitudes", ctypes.c_int64),
                ("n_samples", ctypes.c_int64), ("slices", ctypes.c_int64),
                ("norm", ctypes.c_double), ("footprint_bytes", ctypes.c_double)]


_lib = None
_P = ctypes.c_void_p
_I32, _I64, _U64, _D = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2111_03011_amd/build.py")
        l = ctypes.CDLL(LIB_PATH)
        sig = {
            "tnc_last_error": (ctypes.c_char_p, []),
            "tnc_net_create": (_I32, [ctypes.c_int, ctypes.POINTER(_Desc), ctypes.POINTER(_P)]),
            "tnc_net_set_path": (_I32, [_P, _P, _I32, _P]),
            "tnc_net_set_slices": (_I32, [_P, _P, _I32, _P, _I64]),
            "tnc_net_set_slices_wide": (_I32, [_P, _P, _I32, _P, _I64]),
            "tnc_net_set_targets": (_I32, [_P, _P, _I32, _P, _I64]),
            "tnc_plan_create": (_I32, [_P, ctypes.c_int, _I32, ctypes.POINTER(_P)]),
            "tnc_plan_workspace_bytes": (_I32, [_P, ctypes.POINTER(_U64)]),
            "tnc_plan_stats": (_I32, [_P, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_I32)]),
            "tnc_plan_work": (_I32, [_P, _I64, _I64, ctypes.POINTER(_D)]),
            "tnc_contract": (_I32, [_P, _P, _U64, _P, _P, ctypes.POINTER(_D)]),
            "tnc_contract_range": (_I32, [_P, _P, _U64, _P, _P, _I64, _I64, _I32]),
            "tnc_sample": (_I32, [_P, _P, _U64, _P, _U64, _I64, _P, _P]),
            "tnc_sample_metropolis": (_I32, [_P, _P, _U64, _P, _U64, _I64, _I32, _P, _P]),
            "tnc_sample_frugal": (_I32, [_P, _P, _U64, _P, _U64, _I64, _D, _I32, _P, _P]),
            "tnc_sample_noalloc": (_I32, [_P, _P, _U64, _I64, _P, _P]),
            "tnc_plan_destroy": (_I32, [_P]),
            "tnc_net_destroy": (_I32, [_P]),
            "tnc_plan_batch_slices": (_I32, [_P, ctypes.POINTER(_I32)]),
            "tnc_plan_autotune": (_I32, [_P, _P, _U64, _P, _I32, ctypes.POINTER(_I32)]),
            "tnc_plan_n_launches": (_I32, [_P, ctypes.POINTER(_I32)]),
            "tnc_plan_launch_timing": (_I32, [_P, _I32, ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int64)]),
            "tnc_plan_launch_info": (_I32, [_P, _I32, ctypes.POINTER(StepInfo)]),
            "tnc_plan_set_timing": (_I32, [_P, _I32]),
            "tnc_plan_timing": (_I32, [_P, _P, _P, _P, _P, _I32]),
            "tnc_server_create": (_I32, [ctypes.c_int, _P, _U64, _I32, _I32, ctypes.POINTER(_P)]),
            "tnc_server_submit": (_I32, [_P, _P, ctypes.c_int, _I32, _I64, _U64, ctypes.POINTER(_U64)]),
            "tnc_server_poll": (_I32, [_P, _U64, _P, _P, ctypes.POINTER(RequestInfo)]),
            "tnc_server_pending": (_I32, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32)]),
            "tnc_server_destroy": (_I32, [_P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def _check(status: int) -> None:
    if status != TNC_OK:
        raise TncError(status, lib().tnc_last_error().decode())


def _arr(x, dtype):
    a = np.ascontiguousarray(np.asarray(x, dtype=dtype))
    return a, a.ctypes.data_as(ctypes.c_void_p)


def tnc_net_create(device: int, n_qubits: int, ranks, labels, data, out_label) -> int:
    r, rp = _arr(ranks, np.int32)
    lb, lp = _arr(labels if len(labels) else np.zeros(0), np.int32)
    d = np.ascontiguousarray(np.asarray(data, dtype=np.complex128)).view(np.float64)
    o, op = _arr(out_label if len(out_label) else np.zeros(0), np.int32)
    desc = _Desc(n_qubits, len(r), rp, lp, d.ctypes.data_as(ctypes.c_void_p), op)
    h = _P()
    _check(lib().tnc_net_create(device, ctypes.byref(desc), ctypes.byref(h)))
    return h.value


def tnc_net_set_path(net: int, pairs, out_orders=None) -> None:
    p, pp = _arr(np.asarray(pairs).reshape(-1) if len(pairs) else np.zeros(0), np.int32)
    if out_orders is not None:
        raise TncError(TNC_E_UNSUPPORTED, "explicit result orders are not supported")
    _check(lib().tnc_net_set_path(net, pp, len(p) // 2, None))


def tnc_net_set_slices(net: int, sliced_labels, slice_ids) -> None:
    s, sp = _arr(sliced_labels if len(sliced_labels) else np.zeros(0), np.int32)
    i, ip = _arr(slice_ids, np.uint64)
    _check(lib().tnc_net_set_slices(net, sp, len(s), ip, len(i)))


def tnc_net_set_slices_wide(net: int, sliced_labels, slice_ids) -> None:
    """slice_ids: Python ints below 2^127 (split into two 64-bit words here)."""
    s, sp = _arr(sliced_labels if len(sliced_labels) else np.zeros(0), np.int32)
    words = np.array([[int(x) & ((1 << 64) - 1), int(x) >> 64] for x in slice_ids], dtype=np.uint64)
    w, wp = _arr(words.reshape(-1), np.uint64)
    _check(lib().tnc_net_set_slices_wide(net, sp, len(s), wp, len(words)))


def set_slices_any(net: int, sliced_labels, slice_ids) -> None:
    if len(sliced_labels) <= 63:
        tnc_net_set_slices(net, sliced_labels, np.asarray([int(x) for x in slice_ids], np.uint64))
    else:
        tnc_net_set_slices_wide(net, sliced_labels, slice_ids)


def tnc_net_set_targets(net: int, open_qubits, closed_bits) -> None:
    o, op = _arr(open_qubits if len(open_qubits) else np.zeros(0), np.int32)
    c, cp = _arr(closed_bits, np.uint64)
    _check(lib().tnc_net_set_targets(net, op, len(o), cp, len(c)))


def tnc_plan_create(net: int, precision: int = TNC_C64, max_batch_slices: int = 1) -> int:
    h = _P()
    _check(lib().tnc_plan_create(net, precision, max_batch_slices, ctypes.byref(h)))
    return h.value


def tnc_plan_workspace_bytes(plan: int) -> int:
    b = _U64()
    _check(lib().tnc_plan_workspace_bytes(plan, ctypes.byref(b)))
    return b.value


def tnc_plan_stats(plan: int):
    f, b, n = _D(), _D(), _I32()
    _check(lib().tnc_plan_stats(plan, ctypes.byref(f), ctypes.byref(b), ctypes.byref(n)))
    return f.value, b.value, n.value


def tnc_plan_work(plan: int, first: int, count: int) -> float:
    f = _D()
    _check(lib().tnc_plan_work(plan, first, count, ctypes.byref(f)))
    return f.value


def tnc_contract(plan: int, ws: int, ws_bytes: int, stream: int, amps: int, want_norm: bool = False):
    norm = _D()
    _check(lib().tnc_contract(plan, ws, ws_bytes, stream, amps,
                              ctypes.byref(norm) if want_norm else None))
    return norm.value if want_norm else None


def tnc_contract_range(plan: int, ws: int, ws_bytes: int, stream: int, amps: int,
                       first: int, count: int, accumulate: bool) -> None:
    _check(lib().tnc_contract_range(plan, ws, ws_bytes, stream, amps, first, count,
                                    1 if accumulate else 0))


def tnc_sample(plan: int, ws: int, ws_bytes: int, amps: int, seed: int, n_samples: int,
               stream: int) -> np.ndarray:
    out = np.zeros(n_samples, dtype=np.uint64)
    _check(lib().tnc_sample(plan, ws, ws_bytes, amps, seed & ((1 << 64) - 1), n_samples,
                            out.ctypes.data_as(ctypes.c_void_p), stream))
    return out


def tnc_sample_metropolis(plan: int, ws: int, ws_bytes: int, amps: int, seed: int,
                          n_samples: int, steps: int, stream: int) -> np.ndarray:
    out = np.zeros(n_samples, dtype=np.uint64)
    _check(lib().tnc_sample_metropolis(plan, ws, ws_bytes, amps, seed & ((1 << 64) - 1),
                                       n_samples, steps, out.ctypes.data_as(ctypes.c_void_p),
                                       stream))
    return out


def tnc_sample_frugal(plan: int, ws: int, ws_bytes: int, amps: int, seed: int, n_samples: int,
                      m: float, max_trials: int, stream: int) -> np.ndarray:
    out = np.zeros(n_samples, dtype=np.uint64)
    _check(lib().tnc_sample_frugal(plan, ws, ws_bytes, amps, seed & ((1 << 64) - 1), n_samples,
                                   float(m), max_trials, out.ctypes.data_as(ctypes.c_void_p),
                                   stream))
    return out


def tnc_sample_noalloc(plan: int, amps: int, seed: int, n_samples: int, stream: int) -> np.ndarray:
    out = np.zeros(n_samples, dtype=np.uint64)
    _check(lib().tnc_sample_noalloc(plan, amps, seed & ((1 << 64) - 1), n_samples,
                                    out.ctypes.data_as(ctypes.c_void_p), stream))
    return out


def tnc_plan_destroy(plan: int) -> None:
    _check(lib().tnc_plan_destroy(plan))


def tnc_net_destroy(net: int) -> None:
    _check(lib().tnc_net_destroy(net))


def tnc_plan_batch_slices(plan: int) -> int:
    b = _I32()
    _check(lib().tnc_plan_batch_slices(plan, ctypes.byref(b)))
    return b.value


def tnc_plan_autotune(plan: int, ws: int, ws_bytes: int, stream: int, reps: int = 3) -> int:
    n = _I32()
    _check(lib().tnc_plan_autotune(plan, ws, ws_bytes, stream, reps, ctypes.byref(n)))
    return n.value


def tnc_plan_n_launches(plan: int) -> int:
    n = _I32()
    _check(lib().tnc_plan_n_launches(plan, ctypes.byref(n)))
    return n.value


def tnc_plan_launch_info(plan: int, i: int) -> StepInfo:
    s = StepInfo()
    _check(lib().tnc_plan_launch_info(plan, i, ctypes.byref(s)))
    return s


def tnc_plan_set_timing(plan: int, enable: bool) -> None:
    _check(lib().tnc_plan_set_timing(plan, 1 if enable else 0))


def tnc_plan_timing(plan: int, reset: bool = False):
    nk = len(KIND_NAMES)
    ms = np.zeros(nk)
    by = np.zeros(nk)
    fl = np.zeros(nk)
    n = np.zeros(nk, dtype=np.int64)
    _check(lib().tnc_plan_timing(plan, ms.ctypes.data_as(_P), by.ctypes.data_as(_P),
                                 fl.ctypes.data_as(_P), n.ctypes.data_as(_P), 1 if reset else 0))
    return {KIND_NAMES[k]: {"ms": float(ms[k]), "bytes": float(by[k]), "flops": float(fl[k]),
                            "launches": int(n[k])} for k in range(nk)}


def tnc_plan_launch_timing(plan: int, i: int):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().tnc_plan_launch_timing(plan, i, ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def tnc_server_create(device: int, arena: int, arena_bytes: int, max_slots: int,
                      chunk_batches: int) -> int:
    h = _P()
    _check(lib().tnc_server_create(device, arena, arena_bytes, max_slots, chunk_batches,
                                   ctypes.byref(h)))
    return h.value


def tnc_server_submit(server: int, net: int, precision: int, max_batch_slices: int,
                      n_samples: int, seed: int) -> int:
    rid = _U64()
    _check(lib().tnc_server_submit(server, net, precision, max_batch_slices, n_samples,
                                   seed & ((1 << 64) - 1), ctypes.byref(rid)))
    return rid.value


def tnc_server_poll(server: int, request_id: int, amps: np.ndarray | None,
                    bits: np.ndarray | None):
    """Returns (status, RequestInfo); status TNC_E_BUSY while the request runs.  Other
    non-zero statuses raise."""
    info = RequestInfo()
    st = lib().tnc_server_poll(server, request_id,
                               amps.ctypes.data_as(_P) if amps is not None else None,
                               bits.ctypes.data_as(_P) if bits is not None else None,
                               ctypes.byref(info))
    if st not in (TNC_OK, TNC_E_BUSY):
        raise TncError(st, lib().tnc_last_error().decode())
    return st, info


def tnc_server_pending(server: int):
    q, r = _I32(), _I32()
    _check(lib().tnc_server_pending(server, ctypes.byref(q), ctypes.byref(r)))
    return q.value, r.value


def tnc_server_destroy(server: int) -> None:
    _check(lib().tnc_server_destroy(server))
