"""ctypes declarations of libdiffpower.so (see include/diffpower.h).

Loading fails loudly when the library has not been built: there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdiffpower.so")

_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_st = ctypes.c_int

DP_OK, DP_E_INVALID, DP_E_CYCLE, DP_E_OOM, DP_E_HIP, DP_E_UNSUPPORTED, DP_E_STATE, DP_E_BUDGET, \
    DP_E_NOTFOUND = 0, -1, -2, -3, -4, -5, -6, -7, -8
DP_MODELED, DP_HYBRID, DP_FROZEN_BETA = 0, 1, 2
DP_CELL_BASE = 16
DP_BETA_LOCAL, DP_BETA_STE = 0, 1
DP_SCHED_AUTO, DP_SCHED_LEVEL, DP_SCHED_GRAPH, DP_SCHED_PERSISTENT = 0, 1, 2, 3
DP_Q_FWD, DP_Q_FWD_BWD = 0, 1

STATUS_NAMES = {0: "DP_OK", -1: "DP_E_INVALID", -2: "DP_E_CYCLE", -3: "DP_E_OOM",
                -4: "DP_E_HIP", -5: "DP_E_UNSUPPORTED", -6: "DP_E_STATE", -7: "DP_E_BUDGET",
                -8: "DP_E_NOTFOUND"}


class Netlist(ctypes.Structure):
    _fields_ = [("n_pi", _i32), ("n_gates", _i32), ("op", _p), ("fanin_ptr", _p), ("fanin", _p)]


class Params(ctypes.Structure):
    _fields_ = [("vdd", ctypes.c_double), ("fclk", ctypes.c_double),
                ("energy_factor", ctypes.c_double), ("beta_min", ctypes.c_double),
                ("beta_max", ctypes.c_double), ("mode", _i32), ("beta_grad", _i32),
                ("n_sim", _i64), ("seed", _u64)]


class DesignInfo(ctypes.Structure):
    _fields_ = [("n_pi", _i32), ("n_gates", _i32), ("n_nets", _i32), ("depth", _i32),
                ("n_edges", _i64), ("max_level_width", _i32), ("reserved", _i32),
                ("device_bytes", _i64)]


class FwdOut(ctypes.Structure):
    _fields_ = [("sp", _p), ("tr", _p), ("sp_acc", _p), ("tr_acc", _p), ("beta", _p),
                ("tr_hyb", _p), ("ones", _p), ("toggles", _p), ("power", _p),
                ("on_device", _i32)]


class Profile(ctypes.Structure):
    _fields_ = [("sim_ms", ctypes.c_double), ("sim_launches", _i64), ("sim_bytes", ctypes.c_double),
                ("sp_ms", ctypes.c_double), ("sp_launches", _i64), ("sp_bytes", ctypes.c_double),
                ("bwd_ms", ctypes.c_double), ("bwd_launches", _i64), ("bwd_bytes", ctypes.c_double),
                ("stim_ms", ctypes.c_double), ("stim_launches", _i64)]


class Query(ctypes.Structure):
    _fields_ = [("design_id", _i32), ("kind", _i32), ("pi_prob", _p), ("cap_scale", _p),
                ("power", _p), ("dpower_dpi", _p)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", _i64), ("completed", _i64), ("device_steps", _i64),
                ("busy_s", ctypes.c_double), ("peak_slot_bytes", _i64), ("max_inflight", _i32),
                ("reserved", _i32), ("lanes_created", _i64), ("lanes_freed", _i64),
                ("memory_waits", _i64)]


# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "dp_params_default": (None, [_p]),
    "dp_last_error": (ctypes.c_char_p, []),
    "dp_version": (ctypes.c_char_p, []),
    "dp_ctx_create": (_st, [_i32, _p, _p]),
    "dp_ctx_set_stream": (_st, [_p, _p]),
    "dp_ctx_synchronize": (_st, [_p]),
    "dp_ctx_destroy": (None, [_p]),
    "dp_compile": (_st, [_p, _p, _p]),
    "dp_compile_cells": (_st, [_p, _p, _i32, _p, _p]),
    "dp_compile_library": (_st, [_p, _p, _i32, _p, _p, _p]),
    "dp_design_cell_logic": (_st, [_p, _p, _p]),
    "dp_design_info": (_st, [_p, _p]),
    "dp_design_levels": (_st, [_p, _p]),
    "dp_design_destroy": (None, [_p]),
    "dp_eval_create": (_st, [_p, _i32, _i32, _p, _p]),
    "dp_eval_set_params": (_st, [_p, _p]),
    "dp_eval_destroy": (None, [_p]),
    "dp_set_pi_prob": (_st, [_p, _p, _i32]),
    "dp_set_caps": (_st, [_p, _p, _i32]),
    "dp_set_cell_sizes": (_st, [_p, _p, _i32]),
    "dp_set_beta": (_st, [_p, _p, _i32]),
    "dp_set_stimulus": (_st, [_p, _p, _i32]),
    "dp_set_pi_rates": (_st, [_p, _p, _i32]),
    "dp_set_pi_streams": (_st, [_p, _p]),
    "dp_set_pi_fixed": (_st, [_p, _p]),
    "dp_forward": (_st, [_p, _p]),
    "dp_backward": (_st, [_p, _p, _p, _p, _p, _i32]),
    "dp_backward_columns": (_st, [_p, _p, _i32]),
    "dp_forward_backward_columns": (_st, [_p, _p, _p, _i32]),
    "dp_power_virus": (_st, [_p, _i32, ctypes.c_double, _p, _p, _p, _i32]),
    "dp_power_gradients": (_st, [_p, _p, _p, _i32]),
    "dp_forward_static": (_st, [_p, _p, _p, _p, _p, _p, _p, _p]),
    "dp_group_create": (_st, [_p, _p, _i32, _p]),
    "dp_group_run": (_st, [_p, _i32, _p, _p, _i32]),
    "dp_group_configure": (_st, [_p, _i32, _i32]),
    "dp_group_destroy": (None, [_p]),
    "dp_eval_set_schedule": (_st, [_p, _i32, _i64, _i32]),
    "dp_eval_autotune": (_st, [_p, _i32, _i32, _p]),
    "dp_eval_set_sim_streams": (_st, [_p, _i32]),
    "dp_eval_set_sim_columns": (_st, [_p, _i32]),
    "dp_eval_get_schedule": (_st, [_p, _p, _p, _p, _p]),
    "dp_eval_synchronize": (_st, [_p]),
    "dp_eval_set_barrier_timeout": (_st, [_p, ctypes.c_double]),
    "dp_eval_profile": (_st, [_p, _i32]),
    "dp_eval_get_profile": (_st, [_p, _p]),
    "dp_server_create": (_st, [_p, ctypes.c_size_t, _p]),
    "dp_server_configure": (_st, [_p, _i32, _i32]),
    "dp_server_add_design": (_st, [_p, _p, _p, _p, _p]),
    "dp_submit": (_st, [_p, _p, _p]),
    "dp_poll": (_st, [_p, _u64, _p]),
    "dp_wait": (_st, [_p, _u64, _p]),
    "dp_server_get_stats": (_st, [_p, _p]),
    "dp_server_destroy": (None, [_p]),
}

_lib = None


class DiffPowerError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _settle_hip_runtime():
    """Make sure a process holds one HIP runtime.

    The torch wheel ships its own libamdhip64 (soname libamdhip64.so.7) and
    loads it as "libamdhip64.so".  If libdiffpower.so (which needs
    libamdhip64.so.7) loaded the system runtime first, torch would not
    recognise it by that name and would load a second runtime, which then
    finds no GPU.  Importing torch first, when it is installed, lets
    libdiffpower.so bind to the runtime torch already loaded.
    """
    import importlib.util
    if importlib.util.find_spec("torch") is not None:
        import torch  # noqa: F401


def load(path: str = LIB_PATH):
    """Load and declare the library (cached).  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2608_03778_amd.build` "
                          "(hipcc, gfx950) first")
    _settle_hip_runtime()
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int):
    if status != DP_OK:
        raise DiffPowerError(status, load().dp_last_error().decode())
