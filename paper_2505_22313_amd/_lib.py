"""ctypes loader for libdop.so (the HIP library).

The HIP path has no fallback: if the library is missing or cannot be loaded,
every entry point raises.  torch is imported first so that libdop resolves
the same HIP runtime as torch (one runtime per process).
"""

import ctypes
import os
import re

import torch  # noqa: F401  (loads the process's HIP runtime before libdop)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdop.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "dop.h")

DOP_OK = 0
DOP_NOT_READY = 1
DOP_ERR_INVALID_ARG = -1
DOP_ERR_UNSUPPORTED = -2
DOP_ERR_WORKSPACE = -3
DOP_ERR_DEVICE = -4
DOP_ERR_BUDGET = -5
DOP_ERR_NOT_FOUND = -6
DOP_ERR_SHUTDOWN = -7
DOP_ERR_TIMEOUT = -8

DOP_BANDLIMIT = 1
DOP_UPSAMPLE_NEAREST = 0
DOP_UPSAMPLE_LANCZOS3 = 1
DOP_MAX_UPSAMPLE = 16
DOP_SERVE_FIFO = 0
DOP_SERVE_SIZE_AWARE = 1
DOP_SERVE_CHUNKED = 2

DOP_OUT_CROP = 0
DOP_OUT_FULL = 1
DOP_OP_PROPAGATE = 0
DOP_OP_PSF = 1
DOP_OP_PSF_BACKWARD = 2
DOP_NOALLOC_MAX_BYTES = 167772160
DOP_PROBE_READ = 0
DOP_PROBE_WRITE = 1
DOP_PROBE_COPY = 2
DOP_PROBE_INPLACE = 3
DOP_PROBE_PASSC = 4


class DopProblem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("z", ctypes.c_double),
        ("n_lambda", ctypes.c_int32),
        ("lambda_", ctypes.POINTER(ctypes.c_double)),
        ("n_index", ctypes.POINTER(ctypes.c_double)),
        ("weight", ctypes.POINTER(ctypes.c_float)),
        ("out_mode", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("upsample", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("my", ctypes.c_int32),
    ]


class DopServeStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64),
        ("completed", ctypes.c_uint64),
        ("failed", ctypes.c_uint64),
        ("queued", ctypes.c_uint32),
        ("running", ctypes.c_uint32),
        ("arena_bytes", ctypes.c_uint64),
        ("arena_peak", ctypes.c_uint64),
        ("p50_ms", ctypes.c_double),
        ("p99_ms", ctypes.c_double),
        ("mean_ms", ctypes.c_double),
    ]


class DopPassProfile(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 32),
        ("launches", ctypes.c_uint64),
        ("total_ms", ctypes.c_double),
    ]


class DopError(RuntimeError):
    def __init__(self, status, where, detail):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status}): {detail}")


_lib = None

_VP = ctypes.c_void_p
_PROB = ctypes.POINTER(DopProblem)

_SIGNATURES = {
    "dop_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "dop_last_error": (ctypes.c_char_p, []),
    "dop_context_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_VP)]),
    "dop_context_destroy": (ctypes.c_int, [_VP]),
    "dop_workspace_size": (ctypes.c_int, [_VP, _PROB, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "dop_propagate": (ctypes.c_int, [_VP, _PROB, ctypes.c_int, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "dop_psf": (ctypes.c_int, [_VP, _PROB, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "dop_psf_noalloc": (ctypes.c_int, [_VP, _PROB, _VP, _VP, _VP, _VP, _VP]),
    "dop_psf_backward": (ctypes.c_int, [_VP, _PROB, _VP, _VP, _VP, _VP, _VP, _VP, ctypes.c_size_t, _VP]),
    "dop_serve_create": (ctypes.c_int, [_VP, _VP, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_VP)]),
    "dop_serve_create_mock": (ctypes.c_int, [_VP, ctypes.c_size_t, ctypes.c_int, ctypes.c_double,
                                             ctypes.POINTER(_VP)]),
    "dop_serve_submit": (ctypes.c_int, [_VP, _PROB, _VP, _VP, _VP, ctypes.POINTER(ctypes.c_uint64)]),
    "dop_serve_set_policy": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_double]),
    "dop_serve_poll": (ctypes.c_int, [_VP, ctypes.c_uint64]),
    "dop_serve_wait": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.c_double]),
    "dop_serve_latency": (ctypes.c_int, [_VP, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)]),
    "dop_serve_stats_get": (ctypes.c_int, [_VP, ctypes.POINTER(DopServeStats)]),
    "dop_serve_destroy": (ctypes.c_int, [_VP]),
    "dop_upsample": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP, _VP]),
    "dop_upsample_adjoint": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, _VP, _VP,
                                            _VP]),
    "dop_upsample_rect": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, _VP, _VP, _VP]),
    "dop_upsample_adjoint_rect": (ctypes.c_int, [_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                 ctypes.c_int, _VP, _VP, _VP]),
    "dop_probe_bandwidth": (ctypes.c_int, [_VP, ctypes.c_int, _VP, ctypes.c_size_t, ctypes.c_int,
                                           ctypes.POINTER(ctypes.c_size_t), _VP]),
    "dop_profile_enable": (ctypes.c_int, [_VP, ctypes.c_int]),
    "dop_profile_read": (ctypes.c_int, [_VP, ctypes.POINTER(DopPassProfile), ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int)]),
}


def lib():
    """The loaded libdop (loaded on first use); raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"libdop.so not found at {LIB_PATH}: build it first "
                "(python -m paper_2505_22313_amd.build); there is no fallback path")
        handle = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def status_string(status):
    return lib().dop_status_string(int(status)).decode()


def last_error():
    return lib().dop_last_error().decode()


def check(status, where):
    if status != DOP_OK:
        raise DopError(status, where, last_error())
    return status


def header_functions():
    """Names of the functions that include/dop.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dop_[a-z_]+)\s*\(", text)))
