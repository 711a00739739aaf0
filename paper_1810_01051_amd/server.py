"""Python front end of librk's continuous-batching server (include/rk_server.h).

Corpora are torch uint8 tensors resident on the device; requests carry host
pattern lists.  All scheduling, merging, admission and launches happen in
librk's scheduler thread; this module only marshals arguments.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import check
from .search import Context, _mode, check_text, pack_patterns


class Server:
    def __init__(self, ctx: Context, arena_bytes: int = 1 << 30, max_inflight: int = 2,
                 max_step_requests: int = None, max_step_patterns: int = None, mode="screen",
                 use_graphs: bool = True, admission_timeout_s: float = None, request_timeout_s: float = None):
        """Limits left at None keep the library's defaults
        (rk_server_cfg_default)."""
        self.ctx = ctx
        self.lib = ctx.lib
        cfg = _lib.RkServerCfg()
        self.lib.rk_server_cfg_default(ctypes.byref(cfg))
        cfg.arena_bytes = int(arena_bytes)
        cfg.max_inflight = int(max_inflight)
        if max_step_requests is not None:
            cfg.max_step_requests = int(max_step_requests)
        if max_step_patterns is not None:
            cfg.max_step_patterns = int(max_step_patterns)
        cfg.mode = _mode(mode)
        cfg.use_graphs = 1 if use_graphs else 0
        if admission_timeout_s is not None:
            cfg.admission_timeout_s = float(admission_timeout_s)
        if request_timeout_s is not None:
            cfg.request_timeout_s = float(request_timeout_s)
        h = ctypes.c_void_p()
        check(self.lib.rk_server_create(ctx.h, ctypes.byref(cfg), ctypes.byref(h)), ctx.h, "rk_server_create")
        self.h = h
        self.corpora = []  # keep the tensors alive

    def close(self):
        if getattr(self, "h", None):
            self.lib.rk_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_corpus(self, text) -> int:
        check_text(text)
        cid = ctypes.c_uint32()
        st = self.lib.rk_server_add_corpus(self.h, ctypes.c_void_p(text.data_ptr()), text.numel(), ctypes.byref(cid))
        check(st, None, "rk_server_add_corpus")
        self.corpora.append(text)
        return int(cid.value)

    def submit(self, corpus: int, patterns) -> int:
        blob, offs = pack_patterns(patterns)
        rid = ctypes.c_uint64()
        st = self.lib.rk_server_submit(self.h, int(corpus), blob.ctypes.data_as(ctypes.c_void_p),
                                       offs.ctypes.data_as(ctypes.c_void_p), len(patterns), ctypes.byref(rid))
        check(st, None, "rk_server_submit")
        return int(rid.value)

    def _view_to_result(self, rid: int, v: _lib.RkResultView, fetch: bool):
        k = v.k
        offs = np.ctypeslib.as_array(v.offsets, shape=(k + 1,)).copy() if v.offsets else np.zeros(1, np.uint64)
        tot = int(offs[-1])
        res = {"status": v.status, "offsets": offs, "positions_dev": v.positions_dev, "t_submit": v.t_submit,
               "t_start": v.t_start, "t_done": v.t_done, "step": v.step}
        if fetch and v.status == 0:
            pos = np.zeros(max(tot, 1), dtype=np.uint64)
            check(self.lib.rk_server_fetch(self.h, int(rid), pos.ctypes.data_as(ctypes.c_void_p), pos.size), None,
                  "rk_server_fetch")
            res["positions"] = pos[:tot]
        return res

    def poll(self, rid: int, fetch: bool = True):
        v = _lib.RkResultView()
        st = self.lib.rk_server_poll(self.h, int(rid), ctypes.byref(v))
        if st == _lib.RK_EBUSY:
            return None
        check(st, None, "rk_server_poll")
        return self._view_to_result(rid, v, fetch)

    def wait(self, rid: int, timeout: float = 60.0, fetch: bool = True):
        """Blocks until request rid is done; with fetch, its positions are copied
        to a numpy array (they live in device memory until release)."""
        v = _lib.RkResultView()
        st = self.lib.rk_server_wait(self.h, int(rid), float(timeout), ctypes.byref(v))
        if st == _lib.RK_EBUSY:
            raise TimeoutError("request %d not done after %.1fs" % (rid, timeout))
        check(st, None, "rk_server_wait")
        return self._view_to_result(rid, v, fetch)

    def next_done(self, timeout: float = 60.0):
        """Id of the next finished request, in completion order (each once);
        None if none finishes within timeout."""
        rid = ctypes.c_uint64()
        st = self.lib.rk_server_next_done(self.h, float(timeout), ctypes.byref(rid))
        if st == _lib.RK_EBUSY:
            return None
        check(st, None, "rk_server_next_done")
        return int(rid.value)

    def cancel(self, rid: int) -> int:
        return int(self.lib.rk_server_cancel(self.h, int(rid)))

    def release(self, rid: int):
        check(self.lib.rk_server_release(self.h, int(rid)), None, "rk_server_release")

    def drain(self):
        check(self.lib.rk_server_drain(self.h), None, "rk_server_drain")

    def stats(self) -> dict:
        s = _lib.RkServerStats()
        check(self.lib.rk_server_get_stats(self.h, ctypes.byref(s)), None, "rk_server_get_stats")
        return {f: getattr(s, f) for f, _ in _lib.RkServerStats._fields_}

    def reset_stats(self):
        check(self.lib.rk_server_reset_stats(self.h), None, "rk_server_reset_stats")
