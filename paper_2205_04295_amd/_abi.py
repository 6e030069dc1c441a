"""ctypes declarations of the libmrpie C ABI (include/mrpie.h).

Argument marshalling only: every step of the hot path runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrpie.so")

MRPIE_OK = 0
MRPIE_EINVAL = -1
MRPIE_EUNSUPPORTED = -2
MRPIE_EDEVICE = -3
MRPIE_EWORKSPACE = -4
NOALLOC_MAX_BYTES = 16 << 20
STATUS_NONFINITE = 1
STATUS_POS_CLAMPED = 2


class Problem(C.Structure):
    _fields_ = [("H", C.c_int32), ("W", C.c_int32), ("N", C.c_int32), ("M", C.c_int32), ("J", C.c_int32)]


class Params(C.Structure):
    _fields_ = [
        ("alpha_obj", C.c_float), ("alpha_probe", C.c_float), ("beta", C.c_float), ("gamma", C.c_float),
        ("iterations", C.c_int32), ("iter_offset", C.c_int32), ("probe_update_start", C.c_int32),
        ("subpixel", C.c_int32),
        ("refine", C.c_int32), ("refine_start", C.c_int32), ("upsample", C.c_int32), ("xcorr_norm", C.c_int32),
        ("adam_lr", C.c_float), ("adam_b1", C.c_float), ("adam_b2", C.c_float), ("adam_eps", C.c_float),
        ("xcorr_point", C.c_int32), ("propagator", C.c_int32), ("fresnel", C.c_float),
    ]


PARAM_DEFAULTS = dict(alpha_obj=1.0, alpha_probe=1.0, beta=1.0, gamma=1.0, iterations=1, iter_offset=0,
                      probe_update_start=0, subpixel=0, refine=0, refine_start=0, upsample=100,
                      xcorr_norm=0, adam_lr=0.5, adam_b1=0.9, adam_b2=0.999, adam_eps=1e-8,
                      xcorr_point=0, propagator=0, fresnel=0.0)


def make_params(**kw) -> Params:
    d = dict(PARAM_DEFAULTS)
    for k, v in kw.items():
        if k not in d:
            raise KeyError(f"unknown parameter {k!r}")
        d[k] = v
    return Params(**d)


class Job(C.Structure):
    _fields_ = [("problem", Problem), ("obj", C.c_void_p), ("probe", C.c_void_p), ("pos", C.c_void_p),
                ("intens", C.c_void_p), ("err_out", C.c_void_p), ("status", C.c_void_p),
                ("ws", C.c_void_p), ("ws_bytes", C.c_size_t)]


class Tuning(C.Structure):
    _fields_ = [("rows_radix", C.c_int32), ("cols_radix", C.c_int32), ("rows_threads", C.c_int32),
                ("lds_sweep", C.c_int32), ("cols_width", C.c_int32), ("rows_inplace", C.c_int32),
                ("rows_split", C.c_int32)]


class MrpieError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mrpie error {code}: {msg}")
        self.code = code


_P = C.c_void_p
_SIGS = {
    "mrpie_version": (C.c_char_p, []),
    "mrpie_last_error": (C.c_char_p, []),
    "mrpie_validate": (C.c_int, [C.POINTER(Problem), C.POINTER(Params)]),
    "mrpie_workspace_size": (C.c_int, [C.POINTER(Problem), C.POINTER(Params), C.POINTER(C.c_size_t)]),
    "mrpie_rpie": (C.c_int, [C.POINTER(Problem), C.POINTER(Params), _P, _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "mrpie_rpie_noalloc": (C.c_int, [C.POINTER(Problem), C.POINTER(Params), _P, _P, _P, _P, _P, _P, _P, _P]),
    "mrpie_rpie_batched": (C.c_int, [C.c_int32, C.c_void_p, C.POINTER(Params), C.POINTER(Tuning), _P]),
    "mrpie_set_tuning": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(Tuning)]),
    "mrpie_get_tuning": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(Tuning)]),
    "mrpie_tuning_candidates": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(Tuning), C.c_int32]),
    "mrpie_autotune_workspace_size": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                                C.POINTER(C.c_size_t)]),
    "mrpie_autotune": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, _P, C.c_size_t,
                                 C.POINTER(Tuning), C.POINTER(C.c_float), _P]),
    "mrpie_register_workspace_size": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "mrpie_register": (C.c_int, [C.c_int32, C.c_int32, _P, _P, C.c_int32, C.c_int32, _P, _P, _P, C.c_size_t, _P]),
    "mrpie_adam": (C.c_int, [C.c_int32, C.POINTER(Params), C.c_int32, C.c_int32, _P, _P, _P, C.c_int32, _P]),
    "mrpie_grad_workspace_size": (C.c_int, [C.POINTER(Problem), C.POINTER(C.c_size_t)]),
    "mrpie_loss": (C.c_int, [C.POINTER(Problem), C.c_int32, _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "mrpie_adjoint": (C.c_int, [C.POINTER(Problem), C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                C.c_size_t, _P]),
    "mrpie_fft2": (C.c_int, [C.c_int32, C.c_int32, _P, C.c_int32, _P]),
    "mrpie_modulus": (C.c_int, [C.c_int32, C.c_int32, _P, _P, _P]),
    "mrpie_canvas_workspace_size": (C.c_int, [C.c_int32, C.POINTER(C.c_size_t)]),
    "mrpie_canvas": (C.c_int, [C.POINTER(Problem), _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "mrpie_timing_enable": (C.c_int, [C.c_int32]),
    "mrpie_timing_read": (C.c_int, [C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                     C.c_int32]),
}

_lib = None


def exported_symbols():
    return list(_SIGS)


def load():
    """Load libmrpie.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch (when present) carries its own HIP runtime: load it first so the
    # library binds to the same runtime instead of bringing a second one
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2205_04295_amd.build` "
                          "or __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(rc):
    if rc != MRPIE_OK:
        raise MrpieError(rc, load().mrpie_last_error().decode())
    return rc
