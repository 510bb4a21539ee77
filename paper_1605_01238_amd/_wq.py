"""ctypes binding of libwq.so: the C-ABI of include/wq.h with the same names.

Argument marshalling only; every step of the method runs in the HIP library.
Importing this module loads the library and raises if it is missing (no CPU
fallback exists).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwq.so")

WQ_OK, WQ_EINVAL, WQ_EKNOTS, WQ_ESINGULAR, WQ_EGEOM, WQ_ENOSPACE, WQ_EDEVICE, WQ_ESTATE = 0, -1, -2, -3, -4, -5, -6, -7
WQ_MASS, WQ_STIFF = 1, 2
WQ_FP64, WQ_FP32 = 0, 1
WQ_MIN_P, WQ_MAX_P = 2, 6
WQ_STATIC_SCRATCH_BYTES = 64 << 20   # static scratch of wq_assemble_static, per GPU
WQ_BASIS_BSPLINE = 0
WQ_BASIS_NURBS = 1

STATUS_NAMES = {0: "WQ_OK", -1: "WQ_EINVAL", -2: "WQ_EKNOTS", -3: "WQ_ESINGULAR", -4: "WQ_EGEOM",
                -5: "WQ_ENOSPACE", -6: "WQ_EDEVICE", -7: "WQ_ESTATE"}


class wq_sizes_t(C.Structure):
    _fields_ = [("n", C.c_int64 * 3), ("n_qp", C.c_int64 * 3), ("n_rows", C.c_int64),
                ("nnz", C.c_int64), ("n_qp_total", C.c_int64), ("workspace_bytes", C.c_size_t),
                ("value_bytes", C.c_size_t)]


# (name, restype, argtypes) for every entry point declared in include/wq.h
_P = C.c_void_p
SIGNATURES = [
    ("wq_plan_create", C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.POINTER(C.c_double)),
                                 C.c_int, C.POINTER(_P)]),
    ("wq_sizes", C.c_int, [_P, C.POINTER(wq_sizes_t)]),
    ("wq_qpoints", C.c_int, [_P, C.c_int, C.POINTER(C.c_double)]),
    ("wq_bind", C.c_int, [_P, _P, C.c_size_t, _P]),
    ("wq_setup", C.c_int, [_P, _P, _P, _P]),
    ("wq_setup_nurbs", C.c_int, [_P, _P, _P, _P, C.c_int, _P]),
    ("wq_set_coefficient", C.c_int, [_P, _P, _P]),
    ("wq_set_geometry", C.c_int, [_P, _P, _P, _P]),
    ("wq_qp_physical", C.c_int, [_P, _P, _P]),
    ("wq_pattern", C.c_int, [_P, _P, _P, _P]),
    ("wq_assemble", C.c_int, [_P, C.c_int, _P, _P, _P]),
    ("wq_assemble_static", C.c_int, [_P, C.c_int, _P, _P, _P]),
    ("wq_request_bytes", C.c_int, [_P, C.POINTER(C.c_size_t)]),
    ("wq_assemble_request", C.c_int, [_P, _P, C.c_size_t, _P, C.c_int, _P, _P, _P]),
    ("wq_batch_create", C.c_int, [C.c_int, C.POINTER(_P), C.POINTER(_P)]),
    ("wq_batch_sizes", C.c_int, [_P, C.POINTER(C.c_size_t), C.POINTER(C.c_int)]),
    ("wq_batch_bind", C.c_int, [_P, _P, C.c_size_t, C.POINTER(_P), C.POINTER(_P), _P]),
    ("wq_batch_tune", C.c_int, [_P, C.c_int, _P]),
    ("wq_batch_assemble", C.c_int, [_P, C.c_int, C.c_int, _P]),
    ("wq_batch_schedule", C.c_int, [_P, C.c_int, C.POINTER(C.c_int)]),
    ("wq_batch_last_error", C.c_char_p, [_P]),
    ("wq_batch_destroy", None, [_P]),
    ("wq_weights", C.c_int, [_P, C.c_int, C.c_int, _P, _P, _P, _P]),
    ("wq_field", C.c_int, [_P, _P, _P]),
    ("wq_sync", C.c_int, [_P, _P]),
    ("wq_last_error", C.c_char_p, [_P]),
    ("wq_plan_destroy", None, [_P]),
    ("wq_version", C.c_char_p, []),
]


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} (run paper_1605_01238_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()
globals().update({name: getattr(lib, name) for name, _, _ in SIGNATURES})


class WQError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")


def check(status: int, plan=None) -> None:
    """Raise WQError for a failed call; the message is the plan's last error
    (or, without a plan, that of the last failed wq_plan_create)."""
    if status != WQ_OK:
        raise WQError(status, lib.wq_last_error(plan).decode())
