"""ctypes declarations for liblbm.so (the C ABI of include/lbm.h).

Argument marshalling only.  There is no fallback: if the library has not
been built, loading raises.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbm.so")

LBM_OK = 0
LBM_EINVAL = -1
LBM_ENOMEM = -2
LBM_EDEVICE = -3
LBM_EUNSTABLE = -4
LBM_ESTATE = -5

SCHEME = {"moment": 0, "population": 1, "population_aa": 2}
STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
DTYPE_F64 = 0
DTYPE_F32 = 1


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int)]


class Opts(ctypes.Structure):
    _fields_ = [
        ("scheme", ctypes.c_int),
        ("storage", ctypes.c_int),
        ("beta", ctypes.c_double),
        ("sigma", ctypes.c_double),
        ("s_pi", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("device", ctypes.c_int),
        ("check_every", ctypes.c_int),
        ("split", ctypes.c_int),
        ("steps_per_sweep", ctypes.c_int),
        ("nc_A", ctypes.c_double),
        ("nc_hmax", ctypes.c_int),
        ("state_buffers", ctypes.c_void_p * 2),
        ("state_buffer_bytes", ctypes.c_int64),
    ]


class Fields(ctypes.Structure):
    _fields_ = [
        ("base", ctypes.c_void_p),
        ("field_stride", ctypes.c_int64),
        ("dtype", ctypes.c_int),
        ("on_device", ctypes.c_int),
    ]


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} [code {code}]")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Loads liblbm.so; raises if it is missing (build it with build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2301_01622_amd.build` "
                          "or __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    c_int, c_dbl, c_void = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    sigs = {
        "lbm_default_opts": (None, [P(Opts)]),
        "lbm_create": (c_int, [P(c_void), Grid, c_int, c_dbl, c_int, P(Opts)]),
        "lbm_destroy": (c_int, [c_void]),
        "lbm_set_moments": (c_int, [c_void, P(Fields)]),
        "lbm_get_moments": (c_int, [c_void, P(Fields)]),
        "lbm_set_equilibrium": (c_int, [c_void, P(Fields)]),
        "lbm_step": (c_int, [c_void, c_int]),
        "lbm_reduce": (c_int, [c_void, P(c_dbl)]),
        "lbm_memory_info": (c_int, [c_void, P(ctypes.c_int64), P(ctypes.c_int64)]),
        "lbm_state_bytes": (c_int, [c_void, P(ctypes.c_int64)]),
        "lbm_save_state": (c_int, [c_void, c_void]),
        "lbm_load_state": (c_int, [c_void, c_void]),
        "lbm_step_state": (c_int, [c_void, c_void, c_void]),
        "lbm_step_state2": (c_int, [c_void, c_void, c_void, c_void]),
        "lbm_adjoint_step2_stored": (c_int, [c_void, c_void, c_void, c_void, c_void, c_void]),
        "lbm_adjoint_step": (c_int, [c_void, P(Fields), P(Fields), P(Fields), P(c_dbl)]),
        "lbm_equilibrium_moments": (c_int, [c_void, P(Fields), P(Fields)]),
        "lbm_equilibrium_moments_adjoint": (c_int, [c_void, P(Fields), P(Fields), P(Fields)]),
        "lbm_state_bytes_for": (c_int, [Grid, c_int, c_int, P(Opts), P(ctypes.c_int64)]),
        "lbm_adjoint_step_stored": (c_int, [c_void, c_void, c_void, c_void, c_void]),
        "lbm_adjoint_step_stored_noalloc": (c_int, [c_void, c_void, c_void, c_void, c_void]),
        "lbm_costate_bytes": (c_int, [c_void, P(ctypes.c_int64)]),
        "lbm_costate_to_stored": (c_int, [c_void, c_void, c_void]),
        "lbm_costate_from_stored": (c_int, [c_void, c_void, c_void]),
        "lbm_steps_done": (ctypes.c_int64, [c_void]),
        "lbm_steps_per_sweep": (c_int, [c_void]),
        "lbm_strerror": (ctypes.c_char_p, [c_int]),
        "lbm_last_error": (ctypes.c_char_p, [c_void]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int, ctx=None, what: str = "") -> None:
    if rc != LBM_OK:
        lib = load()
        msg = lib.lbm_strerror(rc).decode()
        if ctx:
            detail = lib.lbm_last_error(ctx).decode()
            if detail:
                msg += f": {detail}"
        raise LbmError(rc, f"{what}: {msg}" if what else msg)
