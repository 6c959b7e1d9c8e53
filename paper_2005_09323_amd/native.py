"""ctypes binding of ``libensemble_lbm.so`` (argument marshalling only).

Every entry point of ``include/lbm.h`` is exposed under its own name.  The
library must have been built (``paper_2005_09323_amd.build.build()``); there
is no fallback: a missing library raises at first use.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libensemble_lbm.so")
HEADER = os.path.join(HERE, "..", "include", "lbm.h")

LBM_OK = 0
LBM_EINVAL = -1
LBM_EHIP = -2
LBM_ERANGE = -3
LBM_EUNSUPPORTED = -4
LBM_ENONFINITE = -5


class LbmError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"[{code}] {message}")
        self.code = code


class MemberDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("sq_x0", ctypes.c_int32), ("sq_y0", ctypes.c_int32),
                ("sq_side", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tau", ctypes.c_double), ("force_x", ctypes.c_double)]


class OpenChannelDesc(ctypes.Structure):
    _fields_ = [("u_c", ctypes.c_double), ("grid_x0", ctypes.c_int32), ("grid_bar", ctypes.c_int32),
                ("sponge_x0", ctypes.c_int32), ("outlet_density", ctypes.c_int32),
                ("sponge_tau", ctypes.c_double)]


_P = ctypes.c_void_p
_I = ctypes.c_int32
_U64 = ctypes.c_uint64
_D = ctypes.c_double
_SIG = {
    "lbm_state_floats": (ctypes.c_size_t, [_P, _I]),
    "lbm_create": (ctypes.c_int, [ctypes.POINTER(_P), _P, _I, _P, _P, ctypes.c_size_t, _P, _I, _P, _P]),
    "lbm_destroy": (ctypes.c_int, [_P]),
    "lbm_init": (ctypes.c_int, [_P, _U64, _D]),
    "lbm_init_flow": (ctypes.c_int, [_P, _U64, _D, _D]),
    "lbm_set_observable": (ctypes.c_int, [_P, _D, _D, _D]),
    "lbm_set_active": (ctypes.c_int, [_P, _P]),
    "lbm_step_batch": (ctypes.c_int, [_P, _I]),
    "lbm_drag": (ctypes.c_int, [_P, _I, _I, _P]),
    "lbm_member_state": (ctypes.c_int, [_P, _I, ctypes.POINTER(_P)]),
    "lbm_member_time": (ctypes.c_int, [_P, _I, ctypes.POINTER(_I)]),
    "lbm_set_time": (ctypes.c_int, [_P, _I]),
    "lbm_flags": (ctypes.c_int, [_P, _P]),
    "lbm_set_flags": (ctypes.c_int, [_P, _P]),
    "lbm_set_tile": (ctypes.c_int, [_P, _I]),
    "lbm_tile_count": (_I, []),
    "lbm_face_diagnostics": (ctypes.c_int, [_P, _P]),
    "lbm_set_collision": (ctypes.c_int, [_P, _I, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
    "lbm_launch_steps": (ctypes.c_int, [_P, ctypes.POINTER(_I)]),
    "lbm_set_open_channel": (ctypes.c_int, [_P, _P]),
    "lbm_set_graphs": (ctypes.c_int, [_P, _I]),
    "lbm_autotune": (ctypes.c_int, [_P, _I, ctypes.POINTER(_I)]),
    "lbm_autotune_cached": (ctypes.c_int, [_P, _I, ctypes.c_char_p, ctypes.POINTER(_I)]),
    "lbm_run_count": (ctypes.c_int, [_P, ctypes.POINTER(_I)]),
    "lbm_set_run_rows": (ctypes.c_int, [_P, _P, _I]),
    "lbm_get_run_rows": (ctypes.c_int, [_P, _P, _I, ctypes.POINTER(_I)]),
    "gktl_select_clone": (ctypes.c_int, [_P, _D, _U64, _I, _D, _P, _I, _P, _P]),
    "lbm_set_cloning": (ctypes.c_int, [_P, _I]),
    "lbm_perturb": (ctypes.c_int, [_P, _P, _U64, _I, _D, _P, _I]),
    "lbm_copy_state_out": (ctypes.c_int, [_P, _I, _P]),
    "lbm_copy_state_in": (ctypes.c_int, [_P, _I, _P, _I]),
    "ams_score_kill_branch": (ctypes.c_int, [_P, _I, _I, _I, _U64, _I, _P, _P, _P, _P, _P, _P, _P]),
    "lbm_window_mean": (ctypes.c_int, [_P, _I, _I, _I, _I, _P, _P]),
    "score_net_params": (_I, []),
    "score_net_workspace_bytes": (ctypes.c_size_t, [_I]),
    "score_features": (ctypes.c_int, [_P, _I, _I, _I, _I, _I, _I, _D, _D, _P]),
    "score_features_active": (ctypes.c_int, [_P, _I, _I, _I, _I, _D, _D, _P, _I, _P]),
    "score_net_forward": (ctypes.c_int, [_P, _P, _I, _P, _P, ctypes.c_size_t, _P]),
    "score_net_grad": (ctypes.c_int, [_P, _P, _P, _I, _P, _P, _P, ctypes.c_size_t, _P]),
    "score_net_grad_noalloc": (ctypes.c_int, [_P, _P, _P, _I, _P, _P, _P]),
    "score_net_adam": (ctypes.c_int, [_P, _P, _P, _P, _I, _D, _D, _D, _D, _P]),
    "gktl_rebuild": (ctypes.c_int, [_P, _P, _P, _P, _I, _I, _I, _I, _I, _D, _P, _P, _P, _P]),
    "window_mean_max": (ctypes.c_int, [_P, _I, _I, _I, _P, _P, _P]),
    "tail_probability": (ctypes.c_int, [_P, _P, _I, _P, _I, _P, _P]),
    "gktl_scgf": (ctypes.c_int, [_P, _I, _D, _P, _P]),
    "return_times": (ctypes.c_int, [_P, _I, _D, _D, _P, _P]),
    "ams_probability": (ctypes.c_int, [_P, _I, _I, _P, _P, _I, _P, _P]),
    "ams_learned_score": (ctypes.c_int, [_P, _P, ctypes.c_int64, ctypes.c_float, ctypes.c_float, _P, _P]),
    "lbm_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2005_09323_amd.build.build()")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIG.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def declared_functions() -> list:
    """Names of the functions ``include/lbm.h`` declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_\w+|gktl_\w+|ams_\w+|score_\w+|window_mean_max|tail_probability)\s*\(", text)) - {"lbm_ctx"})


def check(rc: int) -> None:
    if rc != LBM_OK:
        raise LbmError(rc, lib().lbm_last_error().decode())


def member_desc(m) -> MemberDesc:
    """MemberDesc from any object with nx, ny, tau, force_x, square=(x0, y0, side) or None."""
    sq = m.square if m.square is not None else (0, 0, 0)
    return MemberDesc(int(m.nx), int(m.ny), int(sq[0]), int(sq[1]), int(sq[2]), 0,
                      float(m.tau), float(m.force_x))


def desc_array(members):
    arr = (MemberDesc * len(members))()
    for i, m in enumerate(members):
        arr[i] = member_desc(m)
    return arr
