"""ctypes binding of libstokesmg.so (argument marshalling only).

The library is built in-tree by paper_1502_04070_amd.build; importing this
module does not build anything.  If the library is missing, load() raises:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libstokesmg.so")

SMG_OK = 0
STATUS = {0: "ok", -1: "einval", -2: "ehip", -3: "enomem", -4: "esingular",
          1: "noconv", 2: "diverged", 3: "nonfinite", 4: "incompatible"}
SMOOTHERS = {"ne": 0, "uzawa": 1}
DOMAINS = {"square": 0, "l_shape": 1, "union_jack": 2}


class SmgParams(C.Structure):
    _fields_ = [("smoother", C.c_int), ("tau", C.c_double), ("sigma", C.c_double),
                ("nu_pre", C.c_int), ("nu_post", C.c_int), ("gamma", C.c_int), ("n0", C.c_int),
                ("unfused", C.c_int), ("fuse_depth", C.c_int), ("coarse_max_n", C.c_int),
                ("tile_x", C.c_int), ("domain", C.c_int)]


class SmgError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS.get(code, code)} ({code}): {msg}")
        self.code = code


P = C.c_void_p
D = C.c_double
I = C.c_int
# name -> argument types (all return int)
SIGNATURES = {
    "smg_default_params": [C.POINTER(SmgParams)],
    "smg_setup": [I, D, C.POINTER(SmgParams), C.POINTER(P)],
    "smg_destroy": [P],
    "smg_num_levels": [P],
    "smg_level_size": [P, I, C.POINTER(I), C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
    "smg_load": [P, I, P, P, P, P, P],
    "smg_mass": [P, I, I, P, P, P],
    "smg_pressure_mass": [P, I, P, P, P],
    "smg_apply": [P, I, P, P, P, P, P],
    "smg_residual": [P, I, P, P, P, P, P, P, P, P],
    "smg_smooth": [P, I, I, P, P, P, P, P],
    "smg_restrict": [P, I, P, P, P, P, P],
    "smg_prolong_add": [P, I, P, P, P, P, P],
    "smg_coarse_solve": [P, P, P, P, P, P],
    "smg_project_mean": [P, I, P, P],
    "smg_project_dual": [P, I, P, P],
    "smg_cycle": [P, P, P, P, P, P],
    "smg_cycle_f32": [P, P, P, P, P, P],
    "smg_solve": [P, P, P, D, I, P, P, C.POINTER(I), C.POINTER(D), C.POINTER(D), P],
    "smg_error_norm": [P, P, P, P, P, C.POINTER(D), P],
    "smg_solve_error": [P, P, P, P, P, D, I, P, P, C.POINTER(I), C.POINTER(D), P],
    "smg_solve_mixed": [P, P, P, D, I, P, P, C.POINTER(I), C.POINTER(D), C.POINTER(D), P],
    "smg_dot": [P, I, I, P, P, P, P],
    "smg_time_kernel": [P, I, I, C.POINTER(D), P],
    "smg_batch_setup": [I, C.POINTER(I), C.POINTER(D), C.POINTER(SmgParams), C.POINTER(P)],
    "smg_batch_destroy": [P],
    "smg_batch_size": [P],
    "smg_batch_time_kernel": [P, I, I, C.POINTER(D), P],
    "smg_set_damping": [P, I, D, D],
    "smg_get_damping": [P, I, C.POINTER(D), C.POINTER(D)],
    "smg_batch_set_damping": [P, I, I, D, D],
    "smg_implicit_step": [P, P, P, D, I, P, P, C.POINTER(I), C.POINTER(D), P],
    "smg_implicit_step_mixed": [P, P, P, D, I, P, P, C.POINTER(I), C.POINTER(D), P],
    "smg_batch_implicit_step": [P, P, P, D, I, P, P, P, P, P, P],
    "smg_batch_implicit_step_mixed": [P, P, P, D, I, P, P, P, P, P, P],
    "smg_tune": [I, C.POINTER(I), C.POINTER(D), C.POINTER(SmgParams), I, C.POINTER(SmgParams),
                 C.POINTER(D), C.POINTER(SmgParams), C.POINTER(D), I, C.POINTER(I), P],
    "smg_batch_solve": [P, C.POINTER(P), C.POINTER(P), D, I, C.POINTER(P), C.POINTER(P),
                        C.POINTER(I), C.POINTER(D), C.POINTER(I), P],
    "smg_residual_noalloc": [I, D, I, P, P, P, P, P, P, P, P],
    "smg_batch_solve_mixed": [P, C.POINTER(P), C.POINTER(P), D, I, C.POINTER(P), C.POINTER(P),
                              C.POINTER(I), C.POINTER(D), C.POINTER(I), P],
}

_lib = None


def load() -> C.CDLL:
    """Load libstokesmg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not found: build it with `python -m paper_1502_04070_amd.build`")
    lib = C.CDLL(LIB_PATH)
    for name, args in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.smg_last_error.argtypes = []
    lib.smg_last_error.restype = C.c_char_p
    lib.smg_batch_handle.argtypes = [P, I]
    lib.smg_batch_handle.restype = P
    _lib = lib
    return lib


def check(code: int, where: str, soft_ok: bool = False) -> int:
    if code == SMG_OK or (soft_ok and code > 0):
        return code
    msg = load().smg_last_error().decode(errors="replace")
    raise SmgError(code, where, msg)
