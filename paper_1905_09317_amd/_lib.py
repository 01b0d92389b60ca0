"""ctypes declarations for libc2f.so (include/c2f.h).  Loading fails loudly
if the library has not been built: there is no CPU fallback."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libc2f.so")

C2F_OK, C2F_EINVAL, C2F_ENOMEM, C2F_EDEVICE, C2F_ECAPACITY, C2F_ESTATE, C2F_EBUSY, C2F_EIO = (
    0, -1, -2, -3, -4, -5, -6, -7)
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ECAPACITY", -5: "ESTATE",
                -6: "EBUSY", -7: "EIO"}


class WeatherRow(ctypes.Structure):
    _fields_ = [("ffmc", ctypes.c_float), ("bui", ctypes.c_float), ("ws_kmh", ctypes.c_float),
                ("wd_deg_from", ctypes.c_float)]


class SimParams(ctypes.Structure):
    _fields_ = [("landscape_id", ctypes.c_int32), ("weather_id", ctypes.c_int32),
                ("reps", ctypes.c_int32), ("n_periods", ctypes.c_int32),
                ("seed", ctypes.c_uint64),
                ("ros_sigma", ctypes.c_float), ("ros_threshold", ctypes.c_float),
                ("rounding", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("ignition_mode", ctypes.c_int32), ("ignition_cell", ctypes.c_int32),
                ("scenario_mode", ctypes.c_int32), ("scenario", ctypes.c_int32),
                ("rep_offset", ctypes.c_int32), ("ignition_period", ctypes.c_int32),
                ("burn_hours", ctypes.c_int32), ("burnout_ros", ctypes.c_float),
                ("n_ignitions", ctypes.c_int32), ("ignition_list", ctypes.c_void_p),
                ("hfi_min", ctypes.c_float)]


class Outputs(ctypes.Structure):
    _fields_ = [("scar", ctypes.c_void_p), ("arrival_period", ctypes.c_void_p),
                ("arrival_minute", ctypes.c_void_p), ("burn_count", ctypes.c_void_p),
                ("burned_cells", ctypes.c_void_p), ("ignition_cell", ctypes.c_void_p),
                ("scenario", ctypes.c_void_p), ("on_device", ctypes.c_int32)]


class RunStats(ctypes.Structure):
    _fields_ = [("ignitions", ctypes.c_int64), ("entries", ctypes.c_int64),
                ("rate_evals", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("improvements", ctypes.c_int64), ("relaunches", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("continuations", ctypes.c_int64),
                ("kernel_ms", ctypes.c_double), ("block_threads", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("list_capacity", ctypes.c_int64),
                ("rep_order", ctypes.c_int32)]


class TicketInfo(ctypes.Structure):
    _fields_ = [("submit_ms", ctypes.c_double), ("start_ms", ctypes.c_double),
                ("done_ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("batch_requests", ctypes.c_int32), ("batch_reps", ctypes.c_int32),
                ("lane", ctypes.c_int32), ("status", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime under the same SONAME as the system's;
    # loading torch first makes libc2f bind to that one, so torch tensors and
    # streams and this library share a single HIP runtime in the process.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "or python -m paper_1905_09317_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float
    pp = ctypes.POINTER
    sigs = {
        "c2f_create": ([i32, u64, pp(P)], i32),
        "c2f_destroy": ([P], None),
        "c2f_last_error": ([P], ctypes.c_char_p),
        "c2f_set_stream": ([P, P], i32),
        "c2f_load_landscape": ([P, i32, i32, i32, P, P, f32, f32, pp(i32)], i32),
        "c2f_unload_landscape": ([P, i32], i32),
        "c2f_set_weather": ([P, i32, i32, i32, P, pp(i32)], i32),
        "c2f_unset_weather": ([P, i32], i32),
        "c2f_simulate": ([P, pp(SimParams), pp(Outputs)], i32),
        "c2f_simulate_batch": ([P, i32, pp(SimParams), pp(Outputs)], i32),
        "c2f_simulate_noalloc": ([P, pp(SimParams), pp(Outputs)], i32),
        "c2f_count_work": ([P, pp(SimParams), P, P], i32),
        "c2f_eval_ros": ([P, i32, i32, i32, i32, i32, u64, f32, i32, i32, P, P, P, P, P, P, P, P, P], i32),
        "c2f_fbp_coefficients": ([i32, P], i32),
        "c2f_fbp_crown_coefficients": ([i32, P], i32),
        "c2f_set_landscape_fbp": ([P, i32, f32, f32], i32),
        "c2f_set_tuning": ([P, i32, i64], i32),
        "c2f_autotune": ([P, pp(SimParams)], i32),
        "c2f_save_tuning": ([P, ctypes.c_char_p], i32),
        "c2f_load_tuning": ([P, ctypes.c_char_p], i32),
        "c2f_get_stats": ([P, pp(RunStats)], i32),
        "c2f_submit": ([P, pp(SimParams), pp(Outputs), pp(u64)], i32),
        "c2f_poll": ([P, u64, pp(i32)], i32),
        "c2f_wait": ([P, u64], i32),
        "c2f_wait_info": ([P, u64, pp(TicketInfo)], i32),
        "c2f_set_serving": ([P, i32, i32, i32, u64], i32),
        "c2f_get_memory": ([P, pp(u64), pp(u64)], i32),
        "c2f_set_rep_order": ([P, i32], i32),
        "c2f_set_ignition_map": ([P, i32, P], i32),
        "c2f_derive_landscape": ([P, i32, ctypes.c_int64, P, P, P], i32),
        "c2f_compare_scars": ([P, ctypes.c_int64, i32, i32, P, P, i32, P, P, P], i32),
        "c2f_compare_scars_async": ([P, ctypes.c_int64, i32, i32, P, P, P], i32),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


DECLARED = ("c2f_create", "c2f_destroy", "c2f_last_error", "c2f_set_stream", "c2f_load_landscape",
            "c2f_unload_landscape", "c2f_set_weather", "c2f_unset_weather", "c2f_simulate",
            "c2f_simulate_batch", "c2f_simulate_noalloc", "c2f_count_work", "c2f_eval_ros", "c2f_fbp_coefficients", "c2f_fbp_crown_coefficients",
            "c2f_set_landscape_fbp", "c2f_set_tuning",
            "c2f_autotune", "c2f_save_tuning", "c2f_load_tuning", "c2f_get_stats", "c2f_submit", "c2f_poll", "c2f_wait",
            "c2f_wait_info", "c2f_set_serving", "c2f_get_memory", "c2f_set_rep_order",
            "c2f_set_ignition_map", "c2f_derive_landscape", "c2f_compare_scars",
            "c2f_compare_scars_async")
