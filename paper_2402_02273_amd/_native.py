"""ctypes loader for ``libexpint.so`` (the C ABI of ``include/expint.h``).

Argument marshalling only.  There is no fallback: if the library is missing
or fails to load, every call raises.
"""

from __future__ import annotations

import ctypes
import os
import re
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libexpint.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "expint.h")

OK = 0
EINVAL = -1
EUNSUPPORTED = -2
ENOMEM = -3
EHIP = -4
ENONFINITE = -5
ESTATE = -6
EIO = -7
ERROR_NAMES = {
    EINVAL: "EINVAL",
    EUNSUPPORTED: "EUNSUPPORTED",
    ENOMEM: "ENOMEM",
    EHIP: "EHIP",
    ENONFINITE: "ENONFINITE",
    ESTATE: "ESTATE",
    EIO: "EIO",
}

F64, F32 = 0, 1
NOFLUX, DIRICHLET0 = 0, 1
ALGO_AUTO, ALGO_STENCIL_TAYLOR, ALGO_MODAL = 0, 1, 2
MP_NONE, MP_BF16_SPLIT, MP_FP16_SPLIT = 0, 1, 2
SWEEPS_AUTO, SWEEPS_SINGLE, SWEEPS_PAIRS = 0, 1, 2
SCHEME_EXP_EULER, SCHEME_LINEARISED, SCHEME_EXPRK2 = 0, 1, 2
MAX_CLASSES = 8


class ExpIntError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {message}")
        self.code = code


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("h", ctypes.c_double)]


class DField(ctypes.Structure):
    _fields_ = [
        ("labels", ctypes.c_void_p),
        ("n_classes", ctypes.c_int32),
        ("class_D", ctypes.POINTER(ctypes.c_double)),
        ("D", ctypes.c_void_p),
    ]


class LaunchInfo(ctypes.Structure):
    _fields_ = [
        ("sweeps", ctypes.c_int),
        ("pair_ty", ctypes.c_int32),
        ("pair_lp", ctypes.c_int32),
        ("vec", ctypes.c_int32),
        ("bx", ctypes.c_int32),
        ("by", ctypes.c_int32),
        ("rw", ctypes.c_int32),
        ("lp", ctypes.c_int32),
        ("nt", ctypes.c_int32),
        ("modal_dct", ctypes.c_int32),
    ]


class Opts(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int),
        ("tau", ctypes.c_double),
        ("tol", ctypes.c_double),
        ("theta_max", ctypes.c_double),
        ("algo", ctypes.c_int),
        ("mp", ctypes.c_int),
        ("s", ctypes.c_int32),
        ("m", ctypes.c_int32),
        ("check_finite", ctypes.c_int32),
        ("sweeps", ctypes.c_int),
        ("scheme", ctypes.c_int),
        ("stream", ctypes.c_void_p),
    ]


_P = ctypes.c_void_p
_I = ctypes.c_int
_I32 = ctypes.c_int32
_D = ctypes.c_double
_DP = ctypes.POINTER(ctypes.c_double)
_I32P = ctypes.POINTER(ctypes.c_int32)

SIGNATURES = {
    "expint_opts_default": (_I, [ctypes.POINTER(Opts)]),
    "expint_create": (
        _I,
        [ctypes.POINTER(Grid), ctypes.POINTER(DField), _D, _I, ctypes.POINTER(Opts), ctypes.POINTER(_P)],
    ),
    "expint_destroy": (None, [_P]),
    "expint_get_plan": (_I, [_P, _I32P, _I32P, _DP]),
    "expint_get_launch": (_I, [_P, ctypes.POINTER(LaunchInfo)]),
    "expint_set_params": (_I, [_P, _D, _DP, _I32]),
    "expint_apply": (_I, [_P, _P, _P]),
    "expint_rhs": (_I, [_P, _P, _P]),
    "expint_phi1": (_I, [_P, _P, _P]),
    "expint_phi1_lin": (_I, [_P, _P, _P, _P]),
    "expint_phi12": (_I, [_P, _P, _P, _P]),
    "expint_step": (_I, [_P, _P]),
    "expint_advance": (_I, [_P, _P, _I32]),
    "expint_reduce": (_I, [_P, _I32, _P, _P, _DP]),
    "expint_grad": (_I, [_P, _P, _I32, _P, _I32, _DP, _P, _DP, _DP]),
    "expint_vjp": (_I, [_P, _P, _I32, _P, _I32, _P, _DP, _DP]),
    "expint_batch_create": (
        _I,
        [_I32, ctypes.POINTER(Grid), ctypes.POINTER(DField), _DP, _I, ctypes.POINTER(Opts), ctypes.POINTER(_P)],
    ),
    "expint_batch_advance": (_I, [_P, ctypes.POINTER(_P), _I32]),
    "expint_batch_get_plan": (_I, [_P, _I32, _I32P, _I32P, _DP]),
    "expint_batch_destroy": (None, [_P]),
    "expint_get_stream": (_I, [_P, ctypes.POINTER(_P)]),
    "expint_profile": (_I, [_P, _I32, _I32, _DP]),
    "expint_probe_copy": (_I, [_P, _P, ctypes.c_int64, _I32, _I32, _P, _DP]),
    "expint_probe_mfma": (_I, [_I32, _I32, _I32, _P, _P, _DP]),
    "expint_labels_from_intensity": (_I, [_P, _I32, _I32, _I32, _P, _I32, _I32, _I32, _I32, _P, _P]),
    "expint_advance_volumes": (_I, [_P, _P, _I32, _DP]),
    "expint_tumour_size": (_I, [_P, _P, _D, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]),
    "expint_tumour_size_static": (_I, [_P, _I32, _I32, _I32, _I32, _D, ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int64), _P]),
    "expint_write_vtk": (_I, [ctypes.c_char_p, _I32, _I32, _I32, _D, _P, _I, ctypes.c_char_p, _P]),
    "expint_last_error": (ctypes.c_char_p, []),
}

_lib = None
_lock = threading.Lock()


def header_functions(path: str = HEADER):
    """Names of the functions ``include/expint.h`` declares."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(expint_[a-z0-9_]+)\s*\(", text)))


def lib():
    """The loaded library (raises if it is missing)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
            _lib = L
        return _lib


def last_error() -> str:
    msg = lib().expint_last_error()
    return msg.decode() if msg else ""


def check(code: int):
    if code != OK:
        raise ExpIntError(code, last_error())
    return code
