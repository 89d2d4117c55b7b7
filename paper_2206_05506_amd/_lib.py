"""ctypes binding of libpnce.so: the C entry points of include/pnce.h under
the same names, with argument marshalling only (no computation here).

The library must be built in-tree (``python paper_2206_05506_amd/build.py``);
importing this module without it raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# PNCE_LIBRARY may name another build of the library (e.g. a tuned variant).
LIB_PATH = os.environ.get("PNCE_LIBRARY") or os.path.join(_HERE, "libpnce.so")

PNCE_OK = 0
PNCE_W_LAG_ALIAS = 1
PNCE_E_INVALID = -1
PNCE_E_UNSUPPORTED = -2
PNCE_E_NOMEM = -3
PNCE_E_HIP = -4

PNCE_PREC_F32 = 0
PNCE_PREC_F32S = 1
PNCE_PREC_BF16 = 2
PNCE_PREC_F64 = 3
PNCE_PREC_F64ACC = 4
PNCE_PREC_EXACT = 5
PNCE_PREC_EXACT32 = 6

PNCE_LAGS_ADJACENT = 0
PNCE_LAGS_EQ8 = 1

PNCE_FMT_BF16 = 1
PNCE_FMT_F16 = 2
PNCE_FMT_E4M3 = 3

SYMBOLS = ("pnce_create", "pnce_create_ex", "pnce_destroy", "pnce_get_sequence",
           "pnce_get_lags", "pnce_get_feedback", "pnce_get_shape",
           "pnce_estimate", "pnce_pack", "pnce_estimate_packed", "pnce_adjoint",
           "pnce_refine", "pnce_refine_noalloc", "pnce_debias", "pnce_estimate_ls", "pnce_estimate_cp", "pnce_pack_cp",
           "pnce_pack_ws", "pnce_estimate_host",
           "pnce_varlen_create", "pnce_varlen_destroy", "pnce_varlen_estimate",
           "pnce_varlen_estimate_each", "pnce_varlen_tune", "pnce_varlen_get_tuning",
           "pnce_varlen_set_tuning", "pnce_varlen_stats", "pnce_status_string",
           "pnce_last_error")


class pnce_frame_desc(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int), ("N", ctypes.c_int), ("T", ctypes.c_int),
                ("L", ctypes.c_int), ("y_off", ctypes.c_longlong), ("h_off", ctypes.c_longlong)]


class PnceError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libpnce.so not built at {LIB_PATH}; run "
                          "`python paper_2206_05506_amd/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "pnce_create": ([ctypes.POINTER(_P), _I, _I, _I, _I], _I),
        "pnce_create_ex": ([ctypes.POINTER(_P), _I, _I, _I, _I, ctypes.c_uint, _I], _I),
        "pnce_get_lags": ([_P, _P], _I),
        "pnce_get_feedback": ([_P, ctypes.POINTER(ctypes.c_uint)], _I),
        "pnce_destroy": ([_P], _I),
        "pnce_get_sequence": ([_P, _P], _I),
        "pnce_get_shape": ([_P, _P, _P, _P, _P], _I),
        "pnce_estimate": ([_P, _P, _P, _P, _I, _I, _D, _P, _D], _I),
        "pnce_pack": ([_P, _P, _P, _P, _P, _I, _I], _I),
        "pnce_estimate_packed": ([_P, _P, _P, _P, _P, _I, _I, _D], _I),
        "pnce_adjoint": ([_P, _P, _P, _P, _P, _I, _I, _D, _D], _I),
        "pnce_refine": ([_P, _P, _P, _P, _P, _I, _I], _I),
        "pnce_refine_noalloc": ([_P, _P, _P, _P, _I, _I], _I),
        "pnce_debias": ([_P, _P, _P, _I], _I),
        "pnce_estimate_ls": ([_P, _P, _P, _P, _I, _I, _P], _I),
        "pnce_estimate_cp": ([_P, _P, _P, _I, _P, _I, _I, _P], _I),
        "pnce_pack_cp": ([_P, _P, _P, _I, _P, _P, _I, _I], _I),
        "pnce_pack_ws": ([_P, _P, _P, _I, _P, _P, _I, _I, _P, ctypes.c_size_t], _I),
        "pnce_estimate_host": ([_P, _P, _P, _P, _I, _P, _I, _I, _I, _P, ctypes.c_size_t], _I),
        "pnce_varlen_create": ([ctypes.POINTER(_P), ctypes.POINTER(pnce_frame_desc), _I, _I],
                               _I),
        "pnce_varlen_destroy": ([_P], _I),
        "pnce_varlen_estimate": ([_P, _P, _P, _P, _P], _I),
        "pnce_varlen_estimate_each": ([_P, _P, _P, _P, _P], _I),
        "pnce_varlen_tune": ([_P, _P, _P, _P, _P, _I], _I),
        "pnce_varlen_get_tuning": ([_P, _P, _P, _P, _P, _P], _I),
        "pnce_varlen_set_tuning": ([_P, _I, _P, _P, _P, _P], _I),
        "pnce_varlen_stats": ([_P, _P, _P, _P, _P], _I),
        "pnce_status_string": ([_I], ctypes.c_char_p),
        "pnce_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        try:
            fn = getattr(lib, name)
        except AttributeError as e:
            raise ImportError(f"{LIB_PATH} lacks {name}: it is older than its sources; run "
                              "`python paper_2206_05506_amd/build.py`") from e
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def check(status: int, where: str) -> int:
    """Raise PnceError on a negative status; return warnings (> 0) as is."""
    if status < 0:
        detail = lib.pnce_last_error().decode() or lib.pnce_status_string(status).decode()
        raise PnceError(status, where, detail)
    return status


def pnce_create(N: int, T: int, L: int, R: int):
    """Returns (plan handle, status); status may be PNCE_W_LAG_ALIAS."""
    h = _P()
    st = check(lib.pnce_create(ctypes.byref(h), N, T, L, R), "pnce_create")
    return h, st


def pnce_create_ex(N: int, T: int, L: int, R: int, feedback: int, spacing: int):
    """Returns (plan handle, status); status may be PNCE_W_LAG_ALIAS."""
    h = _P()
    st = check(lib.pnce_create_ex(ctypes.byref(h), N, T, L, R, feedback, spacing),
               "pnce_create_ex")
    return h, st


def pnce_get_lags(plan, out_ptr: int) -> int:
    return check(lib.pnce_get_lags(plan, out_ptr), "pnce_get_lags")


def pnce_get_feedback(plan) -> int:
    f = ctypes.c_uint()
    check(lib.pnce_get_feedback(plan, ctypes.byref(f)), "pnce_get_feedback")
    return f.value


def pnce_destroy(plan) -> int:
    return check(lib.pnce_destroy(plan), "pnce_destroy")


def pnce_get_sequence(plan, out_ptr: int) -> int:
    return check(lib.pnce_get_sequence(plan, out_ptr), "pnce_get_sequence")


def pnce_get_shape(plan):
    v = [_I() for _ in range(4)]
    check(lib.pnce_get_shape(plan, *[ctypes.byref(x) for x in v]), "pnce_get_shape")
    return tuple(x.value for x in v)


def pnce_estimate(plan, stream, Y, H, batch, precision, alpha, scales, beta) -> int:
    return check(lib.pnce_estimate(plan, stream, Y, H, batch, precision, alpha, scales, beta),
                 "pnce_estimate")


def pnce_pack(plan, stream, Y, Yq, scales, batch, fmt) -> int:
    return check(lib.pnce_pack(plan, stream, Y, Yq, scales, batch, fmt), "pnce_pack")


def pnce_estimate_packed(plan, stream, Yq, scales, H, batch, fmt, beta) -> int:
    return check(lib.pnce_estimate_packed(plan, stream, Yq, scales, H, batch, fmt, beta),
                 "pnce_estimate_packed")


def pnce_adjoint(plan, stream, G, A, C, batch, precision, alpha, beta) -> int:
    return check(lib.pnce_adjoint(plan, stream, G, A, C, batch, precision, alpha, beta),
                 "pnce_adjoint")


def pnce_refine(plan, stream, y, X, work, batch, steps) -> int:
    return check(lib.pnce_refine(plan, stream, y, X, work, batch, steps), "pnce_refine")


def pnce_refine_noalloc(plan, stream, y, X, batch, steps) -> int:
    return check(lib.pnce_refine_noalloc(plan, stream, y, X, batch, steps),
                 "pnce_refine_noalloc")


def pnce_debias(plan, stream, H, batch) -> int:
    return check(lib.pnce_debias(plan, stream, H, batch), "pnce_debias")


def pnce_estimate_cp(plan, stream, Y_raw, cp, H, batch, precision, scales) -> int:
    return check(lib.pnce_estimate_cp(plan, stream, Y_raw, cp, H, batch, precision, scales),
                 "pnce_estimate_cp")


def pnce_pack_cp(plan, stream, Y_raw, cp, Yq, scales, batch, fmt) -> int:
    return check(lib.pnce_pack_cp(plan, stream, Y_raw, cp, Yq, scales, batch, fmt),
                 "pnce_pack_cp")


def pack_work_bytes(batch: int) -> int:
    """PNCE_PACK_WORK_BYTES(batch) of include/pnce.h."""
    return 4096 * int(batch) + 4


def pnce_pack_ws(plan, stream, Y_raw, cp, Yq, scales, batch, fmt, work, work_bytes) -> int:
    return check(lib.pnce_pack_ws(plan, stream, Y_raw, cp, Yq, scales, batch, fmt, work,
                                  work_bytes), "pnce_pack_ws")


def host_staging_bytes(R: int, N: int, cp: int, chunk: int, precision: int) -> int:
    """PNCE_HOST_STAGING_BYTES(R, N, cp, chunk, precision) of include/pnce.h."""
    return 2 * int(chunk) * int(R) * (int(N) + int(cp)) * (16 if precision == 3 else 8)


def pnce_estimate_host(plan, stream, copy_stream, Y_host, cp, H, frames, chunk, precision,
                       staging, staging_bytes) -> int:
    return check(lib.pnce_estimate_host(plan, stream, copy_stream, Y_host, cp, H, frames, chunk,
                                        precision, staging, staging_bytes),
                 "pnce_estimate_host")


def pnce_estimate_ls(plan, stream, Y, H, batch, precision, scales) -> int:
    return check(lib.pnce_estimate_ls(plan, stream, Y, H, batch, precision, scales),
                 "pnce_estimate_ls")


def pnce_varlen_create(frames, fmt: int):
    """frames: sequence of (R, N, T, L, y_off, h_off). Returns (handle, status)."""
    arr = (pnce_frame_desc * len(frames))(*[pnce_frame_desc(*f) for f in frames])
    h = _P()
    st = check(lib.pnce_varlen_create(ctypes.byref(h), arr, len(frames), fmt),
               "pnce_varlen_create")
    return h, st


def pnce_varlen_destroy(vplan) -> int:
    return check(lib.pnce_varlen_destroy(vplan), "pnce_varlen_destroy")


def pnce_varlen_estimate(vplan, stream, Yq, scales, H) -> int:
    return check(lib.pnce_varlen_estimate(vplan, stream, Yq, scales, H), "pnce_varlen_estimate")


def pnce_varlen_estimate_each(vplan, stream, Yq, scales, H) -> int:
    return check(lib.pnce_varlen_estimate_each(vplan, stream, Yq, scales, H),
                 "pnce_varlen_estimate_each")


def pnce_varlen_tune(vplan, stream, Yq, scales, H, reps: int) -> int:
    return check(lib.pnce_varlen_tune(vplan, stream, Yq, scales, H, reps), "pnce_varlen_tune")


def pnce_varlen_get_tuning(vplan):
    """Returns a list of (N, K, nc, us_per_unit) per class."""
    n = _I()
    check(lib.pnce_varlen_get_tuning(vplan, ctypes.byref(n), None, None, None, None),
          "pnce_varlen_get_tuning")
    N = (_I * n.value)()
    K = (_I * n.value)()
    nc = (_I * n.value)()
    us = (ctypes.c_float * n.value)()
    check(lib.pnce_varlen_get_tuning(vplan, ctypes.byref(n), N, K, nc, us),
          "pnce_varlen_get_tuning")
    return [(N[i], K[i], nc[i], us[i]) for i in range(n.value)]


def pnce_varlen_set_tuning(vplan, entries) -> int:
    n = len(entries)
    N = (_I * n)(*[e[0] for e in entries])
    K = (_I * n)(*[e[1] for e in entries])
    nc = (_I * n)(*[e[2] for e in entries])
    us = (ctypes.c_float * n)(*[e[3] for e in entries])
    return check(lib.pnce_varlen_set_tuning(vplan, n, N, K, nc, us), "pnce_varlen_set_tuning")


def pnce_varlen_stats(vplan):
    nw, nt = _I(), _I()
    mx, mean = ctypes.c_float(), ctypes.c_float()
    check(lib.pnce_varlen_stats(vplan, ctypes.byref(nw), ctypes.byref(nt), ctypes.byref(mx),
                                ctypes.byref(mean)), "pnce_varlen_stats")
    return {"workgroups": nw.value, "tiles": nt.value, "max_cost_us": mx.value,
            "mean_cost_us": mean.value}


def pnce_status_string(status: int) -> str:
    return lib.pnce_status_string(status).decode()


def pnce_last_error() -> str:
    return lib.pnce_last_error().decode()
