"""ctypes binding of the C ABI in include/elbm.h (argument marshalling only).

The shared library paper_2605_01774_amd/libelbm.so must have been built (build.py); there is
no fallback implementation: loading fails with an error if it is missing.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# one library per velocity set, with the same C ABI
LIB_PATHS = {19: os.path.join(_HERE, "libelbm.so"), 27: os.path.join(_HERE, "libelbm27.so")}
LIB_PATH = LIB_PATHS[19]

ELBM_OK = 0
ERRORS = {-1: "EINVAL", -2: "ESHAPE", -3: "ENOTSPD", -4: "EVELOCITY", -5: "EHIP", -6: "ESTATE"}
PRECISIONS = {"f64": 0, "f32": 1, "bf16": 2, "fp16": 3}
BC = {"periodic": 0, "dirichlet": 1}
FLAG_SCALAR_KERNEL = 1
FLAG_REST_FP32 = 2
FLAG_STOCHASTIC_ROUNDING = 4


class ElbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"elbm error {ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class Config(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("bc_x", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("phi_ref", ctypes.c_double), ("eps", ctypes.c_double),
        ("ghost_floor", ctypes.c_double), ("root_rho", ctypes.c_double),
        ("store_scale", ctypes.c_double),
    ]


class Counters(ctypes.Structure):
    _fields_ = [("fallback_nodes", ctypes.c_uint64), ("flagged_nodes", ctypes.c_uint64),
                ("nonfinite", ctypes.c_uint64), ("guard_nodes", ctypes.c_uint64)]


_LIBS = {}

# (name, restype, argtypes) of every exported entry point
_VP = ctypes.c_void_p
_H = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
SIGNATURES = [
    ("elbm_create", ctypes.c_int, [ctypes.POINTER(Config), ctypes.POINTER(_H)]),
    ("elbm_destroy", ctypes.c_int, [_H]),
    ("elbm_set_stream", ctypes.c_int, [_H, _VP]),
    ("elbm_velocity_table", ctypes.c_int, [ctypes.POINTER(ctypes.c_int32), _DP]),
    ("elbm_population_bytes", ctypes.c_int64, [_H]),
    ("elbm_field_plane_bytes", ctypes.c_int64, [_H]),
    ("elbm_bind_populations", ctypes.c_int, [_H, _VP, _I64, _VP, _I64]),
    ("elbm_set_diffusion_uniform", ctypes.c_int, [_H, _DP]),
    ("elbm_set_diffusion_field", ctypes.c_int, [_H, _VP, _I64, _I32, _VP, _I64, ctypes.POINTER(_I64)]),
    ("elbm_set_diffusion_phases", ctypes.c_int, [_H, _VP, _I64, _I32, _I32, _VP, _I64, _VP, _I64,
                                                  ctypes.POINTER(_I64)]),
    ("elbm_set_velocity_uniform", ctypes.c_int, [_H, _DP]),
    ("elbm_set_velocity_field", ctypes.c_int, [_H, _VP, _I64, _VP, _I64, ctypes.POINTER(_I64)]),
    ("elbm_set_source_uniform", ctypes.c_int, [_H, ctypes.c_double]),
    ("elbm_set_source_field", ctypes.c_int, [_H, _VP, _I64, _VP, _I64]),
    ("elbm_clear_source", ctypes.c_int, [_H]),
    ("elbm_set_source_scale", ctypes.c_int, [_H, ctypes.c_double]),
    ("elbm_set_dirichlet", ctypes.c_int, [_H, ctypes.c_double, ctypes.c_double]),
    ("elbm_init_equilibrium", ctypes.c_int, [_H, _VP, _I64, _VP, _I64]),
    ("elbm_step", ctypes.c_int, [_H, ctypes.c_int64]),
    ("elbm_step_record", ctypes.c_int, [_H, _I64, _VP, _I64, _VP, _I64]),
    ("elbm_step_buffers", ctypes.c_int, [_H, _VP, _I64, _I32, _VP, _I64, _VP, _I64, _VP, _I64]),
    ("elbm_read_moments", ctypes.c_int, [_H, _VP, _I64, _VP, _I64]),
    ("elbm_reduce", ctypes.c_int, [_H, _DP]),
    ("elbm_reduce_noalloc", ctypes.c_int, [_H, _VP, _I64]),
    ("elbm_min_population", ctypes.c_int, [_H, _DP]),
    ("elbm_stream_copy", ctypes.c_int, [_H, _VP, _I64, _VP, _I64]),
    ("elbm_get_populations", ctypes.c_int, [_H, _VP, _I64]),
    ("elbm_set_populations", ctypes.c_int, [_H, _VP, _I64]),
    ("elbm_save_state", ctypes.c_int, [_H, _VP, _I64, ctypes.POINTER(_I64), ctypes.POINTER(_I32)]),
    ("elbm_load_state", ctypes.c_int, [_H, _VP, _I64, _I64, _I32]),
    ("elbm_adjoint_step", ctypes.c_int, [_H, _VP, _I64, _I32, _VP, _I64, _VP, _I64, _VP, _I64, _VP, _I64,
                                         _VP, _I64]),
    ("elbm_gradient_workspace_bytes", ctypes.c_int64, [_H, _I64, _I64]),
    ("elbm_forward_record", ctypes.c_int, [_H, _I64, _I64, _VP, _I64]),
    ("elbm_gradient", ctypes.c_int, [_H, _I64, _I64, _VP, _I64, _VP, _I64, _VP, _I64, _VP, _I64, _VP, _I64]),
    ("elbm_tensor_gradient", ctypes.c_int, [_H, _VP, _I64, _I32, _VP, _I64, _VP, _I64]),
    ("elbm_initial_gradient", ctypes.c_int, [_H, _VP, _I64, _VP, _I64, _VP, _I64]),
    ("elbm_get_counters", ctypes.c_int, [_H, ctypes.POINTER(Counters)]),
    ("elbm_reset_counters", ctypes.c_int, [_H]),
    ("elbm_time", ctypes.c_int64, [_H]),
    ("elbm_last_error", ctypes.c_char_p, []),
]


def load(q: int = 19):
    """Load the library of the velocity set D3Q`q` (libelbm.so for 19, libelbm27.so for
    27). No fallback: raises if it has not been built."""
    if q not in LIB_PATHS:
        raise ValueError("q must be 19 or 27")
    if q not in _LIBS:
        path = LIB_PATHS[q]
        if not os.path.exists(path):
            raise RuntimeError(
                f"HIP library not built: {path} is missing (run "
                "`python -c 'import __graft_entry__ as g; g.build()'` or "
                "`python paper_2605_01774_amd/build.py`)")
        lib = ctypes.CDLL(path)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIBS[q] = lib
    return _LIBS[q]


def check(rc: int, lib=None) -> int:
    """Raise ElbmError with the library's message if rc is an error code."""
    if rc < 0:
        msg = (lib if lib is not None else load()).elbm_last_error().decode(errors="replace")
        raise ElbmError(rc, msg)
    return rc


def velocity_table(q: int = 19):
    """(c[Q][3], W[Q]) of the library's population order."""
    import numpy as np
    c = (ctypes.c_int32 * 81)()
    w = (ctypes.c_double * 27)()
    n = check(load(q).elbm_velocity_table(c, w), load(q))
    return np.array(list(c)[:3 * n], dtype=np.int64).reshape(n, 3), np.array(list(w)[:n])
