"""ctypes binding of libpolyspec.so (include/polyspec.h).

Argument marshalling only: every step of the estimator runs in the HIP
library.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpolyspec.so")

PS_OK, PS_E_INVALID_ARG, PS_E_UNSUPPORTED, PS_E_WORKSPACE, PS_E_HIP, PS_E_INTERNAL = range(6)
PS_F32, PS_F64, PS_I16, PS_C64, PS_C128 = 0, 1, 2, 3, 4
PS_EST_KSTAT, PS_EST_NATURAL, PS_EST_C3OPT = 0, 1, 2
PS_WIN_HANN, PS_WIN_HANN_PERIODIC, PS_WIN_ACG = 0, 1, 2
PS_PREC_FP32, PS_PREC_BF16X3, PS_PREC_FP16X2S = 0, 1, 2
PS_SCHED_BATCHED, PS_SCHED_PER_CHUNK = 0, 1
PS_ORDER_S1, PS_ORDER_S2, PS_ORDER_S3, PS_ORDER_S4 = 1 << 1, 1 << 2, 1 << 3, 1 << 4
PS_FLAG_EMPTY, PS_FLAG_NO_ERRBAR = 1, 2

EXPORTED = (
    "ps_plan_create", "ps_plan_destroy", "ps_plan_query", "ps_record_info", "ps_workspace_size",
    "ps_execute", "ps_coefficients", "ps_status_string", "ps_last_error", "ps_abi_version",
    "ps_enumerate_combos", "ps_profile_enable", "ps_profile_read", "ps_graph_create",
    "ps_graph_launch", "ps_graph_destroy", "ps_streamer_create", "ps_streamer_push",
    "ps_streamer_wait", "ps_streamer_destroy", "ps_streamer_create_multi", "ps_streamer_push_multi",
    "ps_plan_get_tuning", "ps_plan_set_tuning", "ps_plan_autotune",
    "ps_sequential_workspace_size", "ps_execute_sequential", "ps_full_plane",
    "ps_stream_begin", "ps_stream_push", "ps_stream_end", "ps_stream_counts", "ps_stream_export_state",
    "ps_stream_import_state", "ps_stream_destroy", "ps_spectra_zscore", "ps_execute_static",
    "ps_record_chunks", "ps_plan_frame_info",
)
PS_STATIC_SCRATCH_BYTES = 256 * 1024 * 1024
PS_TUNE_MAX = 16


class ps_config(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("orders", C.c_uint32), ("n_channels", C.c_int32),
        ("frame_len", C.c_int32), ("n_freq", C.c_int32), ("m", C.c_int32),
        ("f_max", C.c_double), ("dt", C.c_double), ("window_param", C.c_double),
        ("window", C.c_int32), ("precision", C.c_int32), ("schedule", C.c_int32),
        ("n_combos2", C.c_int32), ("n_combos3", C.c_int32), ("n_combos4", C.c_int32),
        ("combos2", C.POINTER(C.c_int8)), ("combos3", C.POINTER(C.c_int8)),
        ("combos4", C.POINTER(C.c_int8)), ("interlaced", C.c_int32), ("estimator", C.c_int32),
        ("complex_signal", C.c_int32), ("s4_shift", C.c_int32), ("frame_len_set", C.c_int32),
    ]


class ps_record(C.Structure):
    _fields_ = [("d_data", C.c_void_p), ("n_samples", C.c_int64), ("channel_stride", C.c_int64),
                ("dtype", C.c_int32), ("frame_len", C.c_int32)]


class ps_output(C.Structure):
    _fields_ = [("d_s2", C.c_void_p), ("d_s2_err", C.c_void_p), ("d_s3", C.c_void_p),
                ("d_s3_err", C.c_void_p), ("d_s4", C.c_void_p), ("d_s4_err", C.c_void_p),
                ("d_s1", C.c_void_p), ("d_s1_err", C.c_void_p)]


class ps_plan_info(C.Structure):
    _fields_ = [
        ("frame_len", C.c_int32), ("n_freq", C.c_int32), ("n_coef", C.c_int32), ("m", C.c_int32),
        ("n_combos2", C.c_int32), ("n_combos3", C.c_int32), ("n_combos4", C.c_int32),
        ("grid", C.c_int32), ("f_max", C.c_double), ("sum_g", C.c_double * 5),
        ("combos2", C.POINTER(C.c_int8)), ("combos3", C.POINTER(C.c_int8)),
        ("combos4", C.POINTER(C.c_int8)),
    ]


class ps_tuning(C.Structure):
    _fields_ = [("tile_group", C.c_int32), ("s3_frame_batch", C.c_int32)]


class ps_tune_report(C.Structure):
    _fields_ = [("n", C.c_int32), ("best", C.c_int32), ("cand", ps_tuning * PS_TUNE_MAX),
                ("ms", C.c_double * PS_TUNE_MAX)]


_lib = None


class PolyspecError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)}: {detail}")


def load() -> C.CDLL:
    """Load the built library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2505_01231_amd.build`")
    # PyTorch ships its own HIP runtime under the same soname as the system
    # one (libamdhip64.so.7).  Whichever is loaded first serves the whole
    # process; torch must get its own, so it is loaded before this library
    # (which then binds to torch's copy: one runtime, shared device memory).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    lib.ps_plan_create.argtypes = [C.POINTER(ps_config), C.POINTER(vp)]
    lib.ps_plan_destroy.argtypes = [vp]
    lib.ps_plan_query.argtypes = [vp, C.POINTER(ps_plan_info)]
    lib.ps_record_info.argtypes = [vp, i64, C.POINTER(i64), C.POINTER(C.c_uint32)]
    lib.ps_workspace_size.argtypes = [vp, C.POINTER(ps_record), i32, C.POINTER(sz)]
    lib.ps_execute.argtypes = [vp, C.POINTER(ps_record), i32, vp, sz, C.POINTER(ps_output), vp]
    lib.ps_coefficients.argtypes = [vp, C.POINTER(ps_record), vp, vp]
    lib.ps_sequential_workspace_size.argtypes = [vp, C.POINTER(ps_record), i64, i64, C.POINTER(sz)]
    lib.ps_execute_sequential.argtypes = [vp, C.POINTER(ps_record), i64, i64, vp, sz, C.POINTER(ps_output), vp]
    lib.ps_full_plane.argtypes = [vp, i32, C.POINTER(C.c_int8), C.POINTER(ps_output), vp, vp, vp]
    lib.ps_enumerate_combos.argtypes = [i32, i32, C.POINTER(C.c_int8), C.POINTER(i32)]
    lib.ps_profile_enable.argtypes = [vp, i32]
    lib.ps_profile_read.argtypes = [vp, C.POINTER(C.c_double), i32]
    lib.ps_graph_create.argtypes = [vp, C.POINTER(ps_record), i32, vp, sz, C.POINTER(ps_output), C.POINTER(vp)]
    lib.ps_graph_launch.argtypes = [vp, vp]
    lib.ps_graph_destroy.argtypes = [vp]
    lib.ps_streamer_create.argtypes = [vp, i64, i32, i32, C.POINTER(vp)]
    lib.ps_streamer_push.argtypes = [vp, vp, C.POINTER(ps_output), vp, C.POINTER(i32)]
    lib.ps_streamer_wait.argtypes = [vp, i32]
    lib.ps_streamer_destroy.argtypes = [vp]
    lib.ps_streamer_create_multi.argtypes = [vp, i64, i32, i32, i32, C.POINTER(vp)]
    lib.ps_streamer_push_multi.argtypes = [vp, vp, i32, C.POINTER(ps_output), vp, C.POINTER(i32)]
    lib.ps_plan_get_tuning.argtypes = [vp, C.POINTER(ps_tuning)]
    lib.ps_plan_set_tuning.argtypes = [vp, C.POINTER(ps_tuning)]
    lib.ps_plan_autotune.argtypes = [vp, C.POINTER(ps_record), i32, vp, sz, C.POINTER(ps_output), i32, vp,
                                     C.POINTER(ps_tune_report)]
    lib.ps_record_chunks.argtypes = [vp, C.POINTER(ps_record), C.POINTER(i64), C.POINTER(C.c_uint32)]
    lib.ps_record_chunks.restype = C.c_int
    lib.ps_plan_frame_info.argtypes = [vp, i32, C.POINTER(ps_plan_info)]
    lib.ps_plan_frame_info.restype = C.c_int
    lib.ps_execute_static.argtypes = [vp, C.POINTER(ps_record), i32, C.POINTER(ps_output), vp]
    lib.ps_execute_static.restype = C.c_int
    lib.ps_stream_begin.argtypes = [vp, i64, i32, C.POINTER(vp)]
    lib.ps_stream_push.argtypes = [vp, vp, i64, i64, vp]
    lib.ps_stream_end.argtypes = [vp, C.POINTER(ps_output), vp]
    lib.ps_stream_counts.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64)]
    lib.ps_stream_export_state.argtypes = [vp, vp, C.POINTER(sz)]
    lib.ps_stream_import_state.argtypes = [vp, vp, sz]
    lib.ps_stream_destroy.argtypes = [vp]
    lib.ps_spectra_zscore.argtypes = [vp, vp, vp, vp, i64, vp, vp]
    for name in ("ps_stream_begin", "ps_stream_push", "ps_stream_end", "ps_stream_counts",
                 "ps_stream_export_state", "ps_stream_import_state", "ps_stream_destroy", "ps_spectra_zscore",
                 "ps_sequential_workspace_size", "ps_execute_sequential", "ps_full_plane",
                 "ps_plan_get_tuning", "ps_plan_set_tuning", "ps_plan_autotune"):
        getattr(lib, name).restype = C.c_int
    for name in ("ps_plan_create", "ps_plan_destroy", "ps_plan_query", "ps_record_info",
                 "ps_workspace_size", "ps_execute", "ps_coefficients", "ps_enumerate_combos",
                 "ps_profile_enable", "ps_profile_read", "ps_graph_create", "ps_graph_launch",
                 "ps_graph_destroy", "ps_streamer_create", "ps_streamer_push", "ps_streamer_wait",
                 "ps_streamer_destroy", "ps_streamer_create_multi", "ps_streamer_push_multi"):
        getattr(lib, name).restype = C.c_int
    lib.ps_status_string.argtypes = [C.c_int]
    lib.ps_status_string.restype = C.c_char_p
    lib.ps_last_error.argtypes = []
    lib.ps_last_error.restype = C.c_char_p
    lib.ps_abi_version.argtypes = []
    lib.ps_abi_version.restype = C.c_int32
    _lib = lib
    return lib


def status_string(s: int) -> str:
    return load().ps_status_string(s).decode()


def last_error() -> str:
    return load().ps_last_error().decode()


def check(status: int, where: str):
    if status != PS_OK:
        raise PolyspecError(status, where, last_error())
