"""ctypes binding of libsketch.so (include/sketch.h).

Argument marshalling only: every step of the sketch runs in the library's HIP
kernels.  torch is imported first so that the library binds to the same HIP
runtime as torch (both use the soname libamdhip64.so.7); torch provides device
memory and streams.  If the library is missing the import fails loudly --
there is no CPU fallback.
"""
import ctypes
import os

import torch  # noqa: F401  (must precede loading libsketch.so)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsketch.so")

SK_OK, SK_EINVAL, SK_ENOMEM, SK_EDEVICE, SK_ESHAPE, SK_EUNSUPPORTED, SK_ESTATE = 0, -1, -2, -3, -4, -5, -6
SK_F64, SK_F32, SK_BF16 = 0, 1, 2
SK_PERSISTENT, SK_WINDOW, SK_ATTP, SK_P5, SK_COD = 0, 1, 2, 3, 4
SK_SHRINK_EXACT, SK_SHRINK_RAND = 0, 1

STATUS_NAMES = {0: "SK_OK", -1: "SK_EINVAL", -2: "SK_ENOMEM", -3: "SK_EDEVICE", -4: "SK_ESHAPE",
                -5: "SK_EUNSUPPORTED", -6: "SK_ESTATE"}


class sketch_config(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32), ("ell", ctypes.c_int32), ("kind", ctypes.c_int32),
        ("shrink", ctypes.c_int32), ("state_dtype", ctypes.c_int32), ("proj_dtype", ctypes.c_int32),
        ("q", ctypes.c_int32), ("oversample", ctypes.c_int32), ("window_N", ctypes.c_int64),
        ("R", ctypes.c_double), ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint64),
        ("device", ctypes.c_int32), ("use_given_stream", ctypes.c_int32), ("hip_stream", ctypes.c_void_p),
        ("amplify_r", ctypes.c_int32), ("amplify_s", ctypes.c_int32), ("sites", ctypes.c_int32),
        ("d_y", ctypes.c_int32), ("theta", ctypes.c_double),
    ]


class sketch_info_t(ctypes.Structure):
    _fields_ = [
        ("rows_seen", ctypes.c_int64), ("fill", ctypes.c_int64), ("shrinks", ctypes.c_int64),
        ("device_bytes", ctypes.c_int64), ("k", ctypes.c_int32), ("levels", ctypes.c_int32),
    ]


class sketch_stage_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("calls", ctypes.c_int64), ("total_ms", ctypes.c_double)]


CLOCK_FN = ctypes.CFUNCTYPE(ctypes.c_double, ctypes.c_void_p)


class sk_server_config(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32), ("max_inflight", ctypes.c_int32), ("memory_budget", ctypes.c_int64),
        ("max_rows_per_tick", ctypes.c_int64), ("hip_stream", ctypes.c_void_p), ("clock", CLOCK_FN),
        ("clock_ctx", ctypes.c_void_p), ("use_given_stream", ctypes.c_int32),
        ("max_shrinks_per_tick", ctypes.c_int32),
    ]


class sk_completion(ctypes.Structure):
    _fields_ = [
        ("ticket", ctypes.c_int64), ("stream", ctypes.c_int64), ("rows", ctypes.c_int64),
        ("arrival", ctypes.c_double), ("launched", ctypes.c_double), ("done", ctypes.c_double),
    ]


class sk_server_stats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("admitted", "waiting", "closed", "bytes_in_use", "ticks",
                                               "batches", "pending_bursts", "inflight", "rows_done")]


SK_STAGE = {"ingest": 1 << 0, "omega": 1 << 1, "gram": 1 << 2, "project": 1 << 3, "cholqr": 1 << 4,
            "core_gemm": 1 << 5, "eig": 1 << 6, "threshold": 1 << 7, "rebuild": 1 << 8, "eig_back": 1 << 9,
            "eig_reduce": 1 << 10}
SK_STAGE_ALL = 0x7FF

EXPORTS = [
    "sketch_config_init", "sketch_create", "sketch_update", "sketch_update_csr", "sketch_query", "sketch_query_at",
    "window_advance", "sketch_merge", "sketch_merge_tree", "sketch_sync", "sketch_destroy",
    "sketch_last_error", "sketch_info", "sketch_set_memory_budget", "sketch_memory_in_use",
    "sketch_update_batch", "sketch_update_batch_noalloc", "sketch_update_csr_batch", "sketch_profile_enable",
    "sketch_profile_read", "window_stats",
    "server_config_init", "server_create", "server_open", "server_submit", "server_tick", "server_poll",
    "server_drain", "server_query", "server_close", "server_stats", "server_now", "server_destroy",
    "sketch_debug_fail_solver", "server_debug_fail_solver",
]

_lib = None


def load():
    """Loads libsketch.so (built by paper_2601_02019_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_02019_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.sketch_config_init.argtypes = [ctypes.POINTER(sketch_config)]
    lib.sketch_create.argtypes = [ctypes.POINTER(sketch_config), ctypes.POINTER(vp)]
    lib.sketch_update.argtypes = [vp, vp, i64, i64, i32, i32]
    lib.sketch_update_csr.argtypes = [vp, vp, vp, vp, i64, i32]
    lib.sketch_query.argtypes = [vp, vp, i32, i32]
    lib.sketch_query_at.argtypes = [vp, i64, vp, i32, i32]
    lib.window_advance.argtypes = [vp, i64]
    lib.sketch_merge.argtypes = [vp, ctypes.POINTER(vp), i32]
    lib.sketch_merge_tree.argtypes = [vp, ctypes.POINTER(vp), i32]
    lib.sketch_sync.argtypes = [vp]
    lib.sketch_destroy.argtypes = [vp]
    lib.sketch_last_error.argtypes = []
    lib.sketch_last_error.restype = ctypes.c_char_p
    lib.sketch_info.argtypes = [vp, ctypes.POINTER(sketch_info_t)]
    lib.sketch_set_memory_budget.argtypes = [i64]
    lib.sketch_memory_in_use.argtypes = []
    lib.sketch_memory_in_use.restype = i64
    lib.sketch_update_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i64),
                                        i32, i32]
    lib.sketch_update_batch_noalloc.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i64),
                                                i32, i32]
    lib.sketch_update_csr_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                            ctypes.POINTER(vp), ctypes.POINTER(i64), i32]
    lib.window_stats.argtypes = [vp, i32, ctypes.POINTER(i64)]
    lib.p5_update.argtypes = [vp, ctypes.POINTER(i32), vp, i64, i64, i32, i32]
    lib.p5_stats.argtypes = [vp, ctypes.POINTER(i64)]
    lib.p5_coordinator.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp, i32]
    lib.cod_update.argtypes = [vp, vp, i64, vp, i64, i64, i32, i32]
    lib.cod_query.argtypes = [vp, vp, vp, i32, i32]
    lib.cod_product.argtypes = [vp, vp, i32]
    lib.sketch_profile_enable.argtypes = [vp, ctypes.c_uint32]
    lib.sketch_profile_read.argtypes = [vp, ctypes.POINTER(sketch_stage_time), i32, ctypes.POINTER(i32)]
    lib.server_config_init.argtypes = [ctypes.POINTER(sk_server_config)]
    lib.server_create.argtypes = [ctypes.POINTER(sk_server_config), ctypes.POINTER(vp)]
    lib.server_open.argtypes = [vp, ctypes.POINTER(sketch_config), ctypes.POINTER(i64)]
    lib.server_submit.argtypes = [vp, i64, vp, i64, i32, ctypes.c_double, ctypes.POINTER(i64)]
    lib.server_tick.argtypes = [vp, ctypes.POINTER(i32)]
    lib.server_poll.argtypes = [vp, ctypes.POINTER(sk_completion), i32, ctypes.POINTER(i32)]
    lib.server_drain.argtypes = [vp]
    lib.server_query.argtypes = [vp, i64, vp, i32, i32]
    lib.server_close.argtypes = [vp, i64]
    lib.server_stats.argtypes = [vp, ctypes.POINTER(sk_server_stats)]
    lib.server_now.argtypes = [vp]
    lib.server_now.restype = ctypes.c_double
    lib.server_destroy.argtypes = [vp]
    lib.sketch_debug_fail_solver.argtypes = [vp]
    lib.server_debug_fail_solver.argtypes = [vp, i64]
    for name in EXPORTS:
        if name not in ("sketch_last_error", "sketch_memory_in_use", "server_now"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class SketchError(RuntimeError):
    def __init__(self, code, where):
        msg = load().sketch_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code, where):
    if code != SK_OK:
        raise SketchError(code, where)
    return code
