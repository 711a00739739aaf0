"""ctypes declarations of librk's C ABI (include/rk.h).

Argument marshalling only: every step of the search runs inside librk.  The
library is loaded from this package directory; if it is missing the import
fails loudly (build it with ``python paper_1810_01051_amd/build.py``).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librk.so")

RK_OK = 0
RK_EINVAL = -1
RK_ENOMEM = -2
RK_EUNSUPPORTED = -3
RK_EDEVICE = -4
RK_ENOSPACE = -5
RK_EBUSY = -6
RK_ECANCELED = -7
RK_ETIMEDOUT = -8
STATUS_NAMES = {0: "RK_OK", -1: "RK_EINVAL", -2: "RK_ENOMEM", -3: "RK_EUNSUPPORTED", -4: "RK_EDEVICE",
                -5: "RK_ENOSPACE", -6: "RK_EBUSY", -7: "RK_ECANCELED", -8: "RK_ETIMEDOUT"}

RK_MODE_AUTO = 0
RK_MODE_EXACT = 1
RK_MODE_SCREEN = 2

RK_OPT_SLAB_CAP = 1
RK_OPT_TILE_CFG = 2
RK_OPT_GRID = 3
RK_OPT_PROFILE = 4
RK_OPT_QUEUE = 5

RK_MAX_M = 1024
RK_STREAM_M = 64

c_u8p = ctypes.POINTER(ctypes.c_uint8)
c_u64p = ctypes.POINTER(ctypes.c_uint64)
c_u32p = ctypes.POINTER(ctypes.c_uint32)
c_void = ctypes.c_void_p


class RkInstance(ctypes.Structure):
    _fields_ = [("text_dev", c_void), ("n", ctypes.c_uint64), ("bytes_host", c_void),
                ("offsets_host", c_void), ("k", ctypes.c_uint32)]


class RkHostResult(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("total", ctypes.c_uint64), ("offsets", c_u64p), ("positions", c_u64p)]


class RkServerCfg(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_uint32),
                ("max_step_requests", ctypes.c_uint32), ("max_step_patterns", ctypes.c_uint32),
                ("mode", ctypes.c_int), ("use_graphs", ctypes.c_int), ("admission_timeout_s", ctypes.c_double),
                ("request_timeout_s", ctypes.c_double)]


class RkResultView(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("k", ctypes.c_uint32), ("offsets", c_u64p), ("positions_dev", c_void),
                ("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("step", ctypes.c_uint64)]


class RkServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("canceled", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("steps", ctypes.c_uint64), ("bytes_scanned", ctypes.c_uint64),
                ("merged_patterns", ctypes.c_uint64), ("request_patterns", ctypes.c_uint64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("busy_s", ctypes.c_double), ("arena_high_water", ctypes.c_uint64),
                ("queue_depth", ctypes.c_uint32), ("inflight", ctypes.c_uint32),
                ("admission_waits", ctypes.c_uint64), ("step_splits", ctypes.c_uint64)]


# name -> (restype, argtypes); the list mirrors include/rk.h and include/rk_server.h
SIGNATURES = {
    "rk_server_cfg_default": (None, [ctypes.POINTER(RkServerCfg)]),
    "rk_server_create": (ctypes.c_int, [c_void, ctypes.POINTER(RkServerCfg), ctypes.POINTER(c_void)]),
    "rk_server_add_corpus": (ctypes.c_int, [c_void, c_void, ctypes.c_uint64, c_u32p]),
    "rk_server_submit": (ctypes.c_int, [c_void, ctypes.c_uint32, c_void, c_void, ctypes.c_uint32, c_u64p]),
    "rk_server_poll": (ctypes.c_int, [c_void, ctypes.c_uint64, ctypes.POINTER(RkResultView)]),
    "rk_server_wait": (ctypes.c_int, [c_void, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(RkResultView)]),
    "rk_server_cancel": (ctypes.c_int, [c_void, ctypes.c_uint64]),
    "rk_server_release": (ctypes.c_int, [c_void, ctypes.c_uint64]),
    "rk_server_fetch": (ctypes.c_int, [c_void, ctypes.c_uint64, c_void, ctypes.c_uint64]),
    "rk_server_drain": (ctypes.c_int, [c_void]),
    "rk_server_next_done": (ctypes.c_int, [c_void, ctypes.c_double, ctypes.POINTER(ctypes.c_uint64)]),
    "rk_server_get_stats": (ctypes.c_int, [c_void, ctypes.POINTER(RkServerStats)]),
    "rk_server_reset_stats": (ctypes.c_int, [c_void]),
    "rk_server_destroy": (None, [c_void]),
    "rk_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rk_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(c_void)]),
    "rk_ctx_destroy": (None, [c_void]),
    "rk_ctx_last_error": (ctypes.c_char_p, [c_void]),
    "rk_ctx_set_option": (ctypes.c_int, [c_void, ctypes.c_int, ctypes.c_int64]),
    "rk_tile_cfg_count": (ctypes.c_int, []),
    "rk_tile_cfg": (ctypes.c_int, [ctypes.c_int, c_u32p, c_u32p, c_u32p]),
    "rk_ctx_profile": (ctypes.c_int, [c_void, ctypes.c_int, c_u64p, ctypes.POINTER(ctypes.c_double)]),
    "rk_ctx_profile_reset": (ctypes.c_int, [c_void]),
    "rk_hash": (ctypes.c_int, [c_void, c_void, ctypes.c_uint64, c_u64p]),
    "rk_plan_create": (ctypes.c_int, [c_void, c_void, c_void, ctypes.c_uint32, ctypes.c_int,
                                      ctypes.POINTER(c_void)]),
    "rk_plan_destroy": (None, [c_void]),
    "rk_plan_patterns": (ctypes.c_uint32, [c_void]),
    "rk_scratch_size": (ctypes.c_int, [c_void, c_void, ctypes.c_uint64, c_u64p]),
    "rk_count": (ctypes.c_int, [c_void, c_void, c_void, ctypes.c_uint64, c_void, ctypes.c_uint64, c_void, c_u64p,
                                c_void]),
    "rk_work_size": (ctypes.c_int, [c_void, c_void, ctypes.c_uint64, c_u64p]),
    "rk_collect": (ctypes.c_int, [c_void, c_void, c_void, ctypes.c_uint64, c_void, ctypes.c_uint64, c_void,
                                  ctypes.c_uint64, c_void, c_void, ctypes.c_uint64, c_void]),
    "rk_window_hashes": (ctypes.c_int, [c_void, c_void, ctypes.c_uint64, ctypes.c_uint32, c_void,
                                        ctypes.c_uint64, c_void, c_void]),
    "rk_scan_dump": (ctypes.c_int, [c_void, c_void, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, c_void,
                                    ctypes.c_uint64, ctypes.c_int, c_void]),
    "rk_batch_plan_create": (ctypes.c_int, [c_void, ctypes.POINTER(RkInstance), ctypes.c_uint32, ctypes.c_int,
                                            ctypes.POINTER(c_void)]),
    "rk_plan_text_bytes": (ctypes.c_uint64, [c_void]),
    "rk_search_host": (ctypes.c_int, [c_void, c_void, c_void, ctypes.c_uint64, ctypes.c_uint64,
                                      ctypes.POINTER(ctypes.POINTER(RkHostResult))]),
    "rk_search_file": (ctypes.c_int, [c_void, c_void, ctypes.c_char_p, ctypes.c_uint64,
                                      ctypes.POINTER(ctypes.POINTER(RkHostResult))]),
    "rk_host_result_free": (None, [ctypes.POINTER(RkHostResult)]),
    "rk_paper_search": (ctypes.c_int, [c_void, c_void, ctypes.c_uint64, c_void, c_void, ctypes.c_uint32,
                                       ctypes.c_uint32, c_void, c_void, c_void]),
    "rk_paper_scratch_size": (ctypes.c_int, [ctypes.c_uint64, c_u64p]),
    "rk_paper_positions": (ctypes.c_int, [c_void, c_void, ctypes.c_uint64, c_void, ctypes.c_uint64, c_void,
                                          ctypes.c_uint64, c_u64p, c_void]),
    "rk_stream_read": (ctypes.c_int, [c_void, c_void, ctypes.c_uint64, c_void, ctypes.c_uint32, c_void]),
    "rk_search_static": (ctypes.c_int, [c_void, c_void, c_void, ctypes.c_uint64, c_void, c_void, ctypes.c_uint64,
                                        c_u64p, c_void]),
    "rk_static_scratch_bytes": (ctypes.c_uint64, []),
    "rk_autotune": (ctypes.c_int, [c_void, ctypes.c_uint64, c_u32p, ctypes.c_uint32, ctypes.c_char_p]),
    "rk_autotune_load": (ctypes.c_int, [c_void, ctypes.c_char_p]),
    "rk_autotune_choice": (ctypes.c_int, [c_void, ctypes.c_int, ctypes.c_uint32]),
    "rk_autotune_bucket_choice": (ctypes.c_int, [c_void, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load librk.so from the package directory (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("librk.so not found at %s; build it with `python paper_1810_01051_amd/build.py` "
                          "(the HIP path has no fallback)" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class RkError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, str(status)), detail))


def check(status: int, ctx=None, what: str = ""):
    if status != RK_OK:
        detail = ""
        if ctx is not None:
            msg = load().rk_ctx_last_error(ctx)
            detail = msg.decode() if msg else ""
        raise RkError(status, (what + ": " if what else "") + detail)
