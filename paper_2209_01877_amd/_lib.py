"""ctypes binding of libtetdg.so (the C ABI in include/tetdg.h).

Argument marshalling only: every step of the DG path runs in the HIP library.
Importing this module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# TETDG_LIBRARY selects another build of the same library (e.g. one compiled with
# different options); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("TETDG_LIBRARY") or os.path.join(HERE, "libtetdg.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libtetdg.so not found at {LIB_PATH}; build it with paper_2209_01877_amd/build.py "
                      "(or __graft_entry__.build())")

lib = ctypes.CDLL(LIB_PATH)

_i = ctypes.c_int
_i64 = ctypes.c_int64
_p = ctypes.c_void_p
_d = ctypes.c_double
_sz = ctypes.c_size_t
_pp = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "tdg_create": (_i, [_i, _i, _d, _pp]),
    "tdg_destroy": (None, [_p]),
    "tdg_last_error": (ctypes.c_char_p, [_p]),
    "tdg_sizes": (_i, [_p, ctypes.POINTER(_i), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "tdg_mesh_upload": (_i, [_p, _i64, _p, _p, _i64, _p, _p, _i, _p]),
    "tdg_mesh_device_bytes": (_i, [_p, ctypes.POINTER(_sz)]),
    "tdg_mesh_bind": (_i, [_p, _p, _sz, _p]),
    "tdg_set_farfield": (_i, [_p, _p]),
    "tdg_set_flux": (_i, [_p, _i]),
    "tdg_mesh_stats": (_i, [_p, _p]),
    "tdg_state_elems": (_i, [_p, ctypes.POINTER(_i64)]),
    "tdg_state_bytes": (_i, [_p, ctypes.POINTER(_sz)]),
    "tdg_set_state": (_i, [_p, _p, _p, _p]),
    "tdg_get_state": (_i, [_p, _p, _p, _p]),
    "tdg_volume_points": (_i, [_p, _p, _p]),
    "tdg_project": (_i, [_p, _p, _p, _p]),
    "tdg_residual": (_i, [_p, _p, _p, _p]),
    "tdg_rk_step": (_i, [_p, _p, _p, _d, _i, _p]),
    "tdg_rk_step_noalloc": (_i, [_p, _p, _d, _i, _p]),
    "tdg_rk_step_adaptive": (_i, [_p, _p, _p, _d, _i, _p, _p]),
    "tdg_check_state": (_i, [_p, _p, _p, _p]),
    "tdg_set_viscosity": (_i, [_p, _d, _d]),
    "tdg_residual_vjp": (_i, [_p, _p, _p, _p, _p]),
    "tdg_work_bytes": (_i, [_p, ctypes.POINTER(_sz)]),
    "tdg_rk_stage": (_i, [_p, _p, _p, _p, _d, _d, _p]),
    "tdg_residual_vjp_axpy": (_i, [_p, _p, _p, _d, _i, _p, _p, _p, _p]),
    "tdg_wall_pressure": (_i, [_p, _p, _p, _p, _p]),
    "tdg_stable_dt": (_i, [_p, _p, _d, _p, _p]),
    "tdg_sync_check": (_i, [_p, _p]),
    "tdg_debug_tables": (_i, [_i, _i, _p, _sz, ctypes.POINTER(_sz)]),
    "tdg_stream_probe": (_i, [_i, _p, _p, _sz, _p]),
}

for _name, (_res, _args) in _SIGS.items():
    _fn = getattr(lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

STATUS = {0: "TDG_OK", -1: "TDG_ERR_INVALID_ARG", -2: "TDG_ERR_MESH", -3: "TDG_ERR_STATE", -4: "TDG_ERR_HIP",
          -5: "TDG_ERR_UNSUPPORTED", -6: "TDG_ERR_NOMEM"}


class TdgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def check(code: int, ctx=None, what: str = "") -> None:
    if code != 0:
        msg = lib.tdg_last_error(ctx).decode() if ctx else ""
        raise TdgError(code, f"{what}: {msg}" if what else msg)
