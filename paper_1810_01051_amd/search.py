"""Python front end of librk: contexts, plans, single and batched searches.

PyTorch supplies device memory (tensors) and streams only; the search itself
runs in librk's HIP kernels through the C ABI in ``_lib``.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import RK_MODE_EXACT, RK_MODE_SCREEN, RK_MODE_AUTO, check  # noqa: F401

Q = (1 << 61) - 1
D = 256

_MODES = {"auto": RK_MODE_AUTO, "exact": RK_MODE_EXACT, "screen": RK_MODE_SCREEN}


def _mode(mode) -> int:
    if isinstance(mode, str):
        return _MODES[mode]
    return int(mode)


def _stream_handle(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def pack_patterns(patterns):
    pats = [bytes(p) for p in patterns]
    offs = np.zeros(len(pats) + 1, dtype=np.uint64)
    if pats:
        offs[1:] = np.cumsum([len(p) for p in pats], dtype=np.uint64)
    blob = np.frombuffer(b"".join(pats), dtype=np.uint8).copy() if pats else np.zeros(1, np.uint8)
    if blob.size == 0:
        blob = np.zeros(1, np.uint8)
    return blob, offs


class Context:
    """One librk context bound to a HIP device (d = 256, q = 2^61 - 1)."""

    def __init__(self, device: int = 0):
        self.lib = _lib.load()
        self.device = device
        h = ctypes.c_void_p()
        st = self.lib.rk_ctx_create(device, D, Q, ctypes.byref(h))
        check(st, None, "rk_ctx_create(device=%d)" % device)
        self.h = h

    def close(self):
        if self.h:
            self.lib.rk_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_option(self, option: int, value: int):
        check(self.lib.rk_ctx_set_option(self.h, option, int(value)), self.h, "rk_ctx_set_option")

    def profile(self, kernel: int = 3):
        n = ctypes.c_uint64()
        ms = ctypes.c_double()
        check(self.lib.rk_ctx_profile(self.h, kernel, ctypes.byref(n), ctypes.byref(ms)), self.h, "rk_ctx_profile")
        return int(n.value), float(ms.value)

    def profile_reset(self):
        check(self.lib.rk_ctx_profile_reset(self.h), self.h, "rk_ctx_profile_reset")

    def hash(self, s: bytes) -> int:
        buf = np.frombuffer(bytes(s), dtype=np.uint8) if len(s) else np.zeros(1, np.uint8)
        out = ctypes.c_uint64()
        check(self.lib.rk_hash(self.h, buf.ctypes.data_as(ctypes.c_void_p), len(s), ctypes.byref(out)), self.h)
        return int(out.value)

    def autotune(self, n: int, lengths, path: str | None = None):
        arr = (ctypes.c_uint32 * len(lengths))(*lengths)
        check(self.lib.rk_autotune(self.h, int(n), arr, len(lengths), path.encode() if path else None), self.h,
              "rk_autotune")

    def autotune_load(self, path: str):
        check(self.lib.rk_autotune_load(self.h, path.encode()), self.h, "rk_autotune_load")

    def autotune_choice(self, mode, m: int) -> int:
        return int(self.lib.rk_autotune_choice(self.h, _mode(mode), int(m)))

    def autotune_bucket_choice(self, mode, mclass: int, kclass: int) -> int:
        return int(self.lib.rk_autotune_bucket_choice(self.h, _mode(mode), int(mclass), int(kclass)))

    # -------------------------------------------------------------- hashes
    def window_hashes(self, text: torch.Tensor, m: int, xs: torch.Tensor, stream=None) -> torch.Tensor:
        """Hash of text[x : x+m] for every x in xs (int64 tensor on the device)."""
        xs = xs.to(device=text.device, dtype=torch.int64).contiguous()
        out = torch.empty(xs.numel(), dtype=torch.int64, device=text.device)
        check(self.lib.rk_window_hashes(self.h, ctypes.c_void_p(text.data_ptr()), text.numel(), int(m),
                                        ctypes.c_void_p(xs.data_ptr()), xs.numel(),
                                        ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)), self.h,
              "rk_window_hashes")
        return out

    def scan_dump(self, text: torch.Tensor, m: int, stride: int, kernel: int = 0, stream=None) -> torch.Tensor:
        """Hashes of windows x = 0, stride, 2*stride, ... taken from a scan
        kernel's rolling state (kernel 0: the general scan kernel, 1: the
        single-bucket kernel of one-pattern searches)."""
        n = text.numel()
        cnt = 0 if n < m else (n - m) // stride + 1
        out = torch.full((max(cnt, 1),), -1, dtype=torch.int64, device=text.device)
        check(self.lib.rk_scan_dump(self.h, ctypes.c_void_p(text.data_ptr()), n, int(m), int(stride),
                                    ctypes.c_void_p(out.data_ptr()), out.numel(), int(kernel),
                                    _stream_handle(stream)), self.h, "rk_scan_dump")
        return out[:cnt]

    def paper_search(self, text: torch.Tensor, pattern: bytes, threads_per_block: int = 1024, hashes: bool = False,
                     stream=None):
        """The paper's GPU procedure (rk_paper_search): returns the result
        byte array (n - m + 1 entries, 1 at every match) and, with hashes,
        every window's 32-bit shift-add hash (int64 tensor)."""
        pattern = bytes(pattern)
        m = len(pattern)
        n = text.numel()
        nwin = max(n - m + 1, 0)
        flags = torch.empty(max(nwin, 1), dtype=torch.uint8, device=text.device)
        hs = torch.empty(max(nwin, 1), dtype=torch.int32, device=text.device) if hashes else None
        pat_host = np.frombuffer(pattern, np.uint8).copy() if m else np.zeros(1, np.uint8)
        pat_dev = torch.from_numpy(pat_host).to(text.device)
        check(self.lib.rk_paper_search(self.h, ctypes.c_void_p(text.data_ptr()), n,
                                       ctypes.c_void_p(pat_dev.data_ptr()), pat_host.ctypes.data_as(ctypes.c_void_p),
                                       m, int(threads_per_block), ctypes.c_void_p(flags.data_ptr()),
                                       ctypes.c_void_p(hs.data_ptr()) if hs is not None else None,
                                       _stream_handle(stream)), self.h, "rk_paper_search")
        flags = flags[:nwin]
        if hashes:
            return flags, (hs[:nwin].to(torch.int64) & 0xFFFFFFFF)
        return flags

    def paper_positions(self, flags: torch.Tensor, stream=None) -> torch.Tensor:
        """Ascending positions of the nonzero bytes of a paper-mode result array."""
        nf = flags.numel()
        b = ctypes.c_uint64()
        check(self.lib.rk_paper_scratch_size(nf, ctypes.byref(b)), None, "rk_paper_scratch_size")
        scratch = torch.empty(max(int(b.value), 256), dtype=torch.uint8, device=flags.device)
        tot = ctypes.c_uint64()
        cap = 1 << 16
        while True:
            pos = torch.empty(cap, dtype=torch.int64, device=flags.device)
            st = self.lib.rk_paper_positions(self.h, ctypes.c_void_p(flags.data_ptr()), nf,
                                             ctypes.c_void_p(scratch.data_ptr()), scratch.numel(),
                                             ctypes.c_void_p(pos.data_ptr()), cap, ctypes.byref(tot),
                                             _stream_handle(stream))
            if st == _lib.RK_ENOSPACE and tot.value > cap:
                cap = int(tot.value)
                continue
            check(st, self.h, "rk_paper_positions")
            return pos[:int(tot.value)]


class Plan:
    """Preprocessed pattern set (lengths bucketed, hashes and tables on the device)."""

    def __init__(self, ctx: Context, patterns, mode="auto"):
        self.ctx = ctx
        self.lib = ctx.lib
        self.patterns = [bytes(p) for p in patterns]
        self.k = len(self.patterns)
        blob, offs = pack_patterns(self.patterns)
        h = ctypes.c_void_p()
        check(self.lib.rk_plan_create(ctx.h, blob.ctypes.data_as(ctypes.c_void_p),
                                      offs.ctypes.data_as(ctypes.c_void_p), self.k, _mode(mode), ctypes.byref(h)),
              ctx.h, "rk_plan_create")
        self.h = h
        self._scratch = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.rk_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def scratch_size(self, n: int) -> int:
        b = ctypes.c_uint64()
        check(self.lib.rk_scratch_size(self.ctx.h, self.h, int(n), ctypes.byref(b)), self.ctx.h, "rk_scratch_size")
        return int(b.value)

    def work_size(self, total: int) -> int:
        b = ctypes.c_uint64()
        check(self.lib.rk_work_size(self.ctx.h, self.h, int(total), ctypes.byref(b)), self.ctx.h, "rk_work_size")
        return int(b.value)

    def scratch(self, n: int, device) -> torch.Tensor:
        need = self.scratch_size(n)
        if self._scratch is None or self._scratch.numel() < need or self._scratch.device != device:
            self._scratch = torch.empty(max(need, 256), dtype=torch.uint8, device=device)
        return self._scratch

    def count(self, text: torch.Tensor, scratch: torch.Tensor | None = None, stream=None,
              counts: torch.Tensor | None = None) -> int:
        """Count pass; returns the total.  counts (optional, k int64 on the
        device) receives each pattern's number of occurrences."""
        if scratch is None:
            scratch = self.scratch(text.numel(), text.device)
        if counts is not None and (counts.dtype != torch.int64 or counts.numel() < self.k or not counts.is_contiguous()):
            raise ValueError("counts must be a contiguous int64 tensor of k entries")
        tot = ctypes.c_uint64()
        check(self.lib.rk_count(self.ctx.h, self.h, ctypes.c_void_p(text.data_ptr()), text.numel(),
                                ctypes.c_void_p(scratch.data_ptr()), scratch.numel(),
                                ctypes.c_void_p(counts.data_ptr()) if counts is not None else None,
                                ctypes.byref(tot), _stream_handle(stream)), self.ctx.h, "rk_count")
        return int(tot.value)

    def collect(self, text: torch.Tensor, total: int, scratch: torch.Tensor | None = None,
                out: tuple | None = None, stream=None):
        if scratch is None:
            scratch = self.scratch(text.numel(), text.device)
        dev = text.device
        wb = self.work_size(total)
        work = torch.empty(max(wb, 1), dtype=torch.uint8, device=dev) if wb else None
        if out is None:
            offsets = torch.empty(self.k + 1, dtype=torch.int64, device=dev)
            positions = torch.empty(max(total, 1), dtype=torch.int64, device=dev)
        else:
            offsets, positions = out
        check(self.lib.rk_collect(self.ctx.h, self.h, ctypes.c_void_p(text.data_ptr()), text.numel(),
                                  ctypes.c_void_p(scratch.data_ptr()), scratch.numel(),
                                  ctypes.c_void_p(work.data_ptr() if work is not None else 0), wb,
                                  ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(positions.data_ptr()),
                                  positions.numel(), _stream_handle(stream)), self.ctx.h, "rk_collect")
        return offsets, positions[:total]

    def search(self, text: torch.Tensor, stream=None):
        """Returns (offsets int64[k+1], positions int64[total]) on the device."""
        total = self.count(text, stream=stream)
        return self.collect(text, total, stream=stream)

    def search_host(self, text, piece_bytes: int = 256 << 20):
        """Streamed search of a text in host memory (numpy uint8 / bytes) or a
        file (str path), of any length: returns (offsets, positions) as numpy
        uint64 arrays in host memory."""
        res = ctypes.POINTER(_lib.RkHostResult)()
        if isinstance(text, str):
            st = self.lib.rk_search_file(self.ctx.h, self.h, text.encode(), int(piece_bytes), ctypes.byref(res))
        else:
            a = np.ascontiguousarray(np.frombuffer(text, np.uint8) if isinstance(text, (bytes, bytearray)) else text,
                                     dtype=np.uint8)
            st = self.lib.rk_search_host(self.ctx.h, self.h, a.ctypes.data_as(ctypes.c_void_p) if a.size else None,
                                         a.size, int(piece_bytes), ctypes.byref(res))
        check(st, self.ctx.h, "rk_search_host")
        r = res.contents
        try:
            offsets = np.ctypeslib.as_array(r.offsets, shape=(r.k + 1,)).copy()
            positions = (np.ctypeslib.as_array(r.positions, shape=(r.total,)).copy() if r.total
                         else np.zeros(0, np.uint64))
        finally:
            self.lib.rk_host_result_free(res)
        return offsets, positions


def check_text(text: torch.Tensor):
    if text.dtype != torch.uint8 or not text.is_cuda or not text.is_contiguous():
        raise ValueError("text must be a contiguous uint8 CUDA tensor")
    if text.data_ptr() % 16:
        raise ValueError("text must start on a 16-byte boundary")


_default_ctx = {}


def default_context(device: int = 0) -> Context:
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def search(text: torch.Tensor, patterns, mode="auto", ctx: Context | None = None, stream=None):
    """All occurrences of every pattern in text.

    Returns (offsets, positions): int64 device tensors; pattern j's ascending
    positions are positions[offsets[j]:offsets[j+1]]."""
    check_text(text)
    ctx = ctx or default_context(text.device.index or 0)
    plan = Plan(ctx, patterns, mode)
    try:
        return plan.search(text, stream=stream)
    finally:
        plan.close()


def split(offsets, positions):
    o = offsets.cpu().tolist() if isinstance(offsets, torch.Tensor) else list(offsets)
    p = positions.cpu().numpy() if isinstance(positions, torch.Tensor) else np.asarray(positions)
    return [p[o[j]:o[j + 1]] for j in range(len(o) - 1)]


class BatchPlan:
    """Many independent searches scanned by one persistent launch."""

    def __init__(self, ctx: Context, texts, pattern_lists, mode="auto"):
        self.ctx = ctx
        self.lib = ctx.lib
        self.texts = list(texts)
        self.count_inst = len(self.texts)
        self.ks = [len(p) for p in pattern_lists]
        self.k_total = sum(self.ks)
        self._keep = []
        arr = (_lib.RkInstance * max(1, self.count_inst))()
        for i, (t, pats) in enumerate(zip(self.texts, pattern_lists)):
            check_text(t)
            blob, offs = pack_patterns(pats)
            self._keep.append((blob, offs))
            arr[i].text_dev = t.data_ptr()
            arr[i].n = t.numel()
            arr[i].bytes_host = blob.ctypes.data
            arr[i].offsets_host = offs.ctypes.data
            arr[i].k = len(pats)
        h = ctypes.c_void_p()
        check(self.lib.rk_batch_plan_create(ctx.h, arr, self.count_inst, _mode(mode), ctypes.byref(h)), ctx.h,
              "rk_batch_plan_create")
        self.h = h
        self._keep = None
        self.n_total = int(self.lib.rk_plan_text_bytes(self.h))
        self._scratch = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.rk_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def search(self, device=None, stream=None):
        device = device or self.texts[0].device
        b = ctypes.c_uint64()
        check(self.lib.rk_scratch_size(self.ctx.h, self.h, self.n_total, ctypes.byref(b)), self.ctx.h)
        if self._scratch is None or self._scratch.numel() < b.value:
            self._scratch = torch.empty(max(int(b.value), 256), dtype=torch.uint8, device=device)
        sc = self._scratch
        tot = ctypes.c_uint64()
        check(self.lib.rk_count(self.ctx.h, self.h, None, self.n_total, ctypes.c_void_p(sc.data_ptr()), sc.numel(),
                                None, ctypes.byref(tot), _stream_handle(stream)), self.ctx.h, "rk_count(batch)")
        total = int(tot.value)
        wb = ctypes.c_uint64()
        check(self.lib.rk_work_size(self.ctx.h, self.h, total, ctypes.byref(wb)), self.ctx.h)
        work = torch.empty(max(int(wb.value), 1), dtype=torch.uint8, device=device)
        offsets = torch.empty(self.k_total + 1, dtype=torch.int64, device=device)
        positions = torch.empty(max(total, 1), dtype=torch.int64, device=device)
        check(self.lib.rk_collect(self.ctx.h, self.h, None, self.n_total, ctypes.c_void_p(sc.data_ptr()),
                                  sc.numel(), ctypes.c_void_p(work.data_ptr()), int(wb.value),
                                  ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(positions.data_ptr()),
                                  positions.numel(), _stream_handle(stream)), self.ctx.h, "rk_collect(batch)")
        return offsets, positions[:total]

    def split(self, offsets, positions):
        """Per instance, per pattern arrays of positions."""
        lists = split(offsets, positions)
        out, b = [], 0
        for k in self.ks:
            out.append(lists[b:b + k])
            b += k
        return out
