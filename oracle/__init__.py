"""CPU reference oracle for multi-pattern Rabin-Karp search.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and by
the CPU-baseline leg of the benchmark, never by the product package.  It shares
no code with the HIP implementation; only the seeded input generators (the
``rkgen`` package) serve both sides.

The arithmetic lives in ``rk_oracle.c`` (plain C, ``unsigned __int128`` products
reduced with ``%``).  This module only loads it and marshals numpy arrays.

What is computed (Shah & Oza, Sec. 3.1, sequential and GPU pseudo code):
  * ``hash``          -- Horner evaluation h <- h*d + s[i] (mod q) of one string.
  * ``window_hashes`` -- the same hash of chosen text windows, each evaluated
                         from scratch.
  * ``search``        -- Rabin-Karp over every window x in [0, n-m] with the
                         textbook rolling update, hash-set probe and byte check;
                         per-pattern ascending positions.
  * ``search_recompute`` -- the paper's loop: each window hash recomputed.
  * ``brute``         -- the definition: byte comparison at every window.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

D_DEFAULT = 256
Q_DEFAULT = (1 << 61) - 1

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rk_oracle.c")
_LIB = os.path.join(_HERE, "librko.so")

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u64pp = ctypes.POINTER(_u64p)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, -O2) into oracle/librko.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.rko_hash.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        lib.rko_hash.restype = ctypes.c_uint64
        lib.rko_pow.argtypes = [ctypes.c_uint64] * 3
        lib.rko_pow.restype = ctypes.c_uint64
        lib.rko_window_hashes.argtypes = [_u8p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64,
                                          ctypes.c_uint64, _u64p, ctypes.c_uint64, _u64p]
        lib.rko_window_hashes.restype = ctypes.c_int
        lib.rko_search.argtypes = [_u8p, ctypes.c_uint64, _u8p, _u64p, ctypes.c_uint32,
                                   ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, _u64pp, _u64pp]
        lib.rko_search.restype = ctypes.c_int
        lib.rko_search_recompute.argtypes = [_u8p, ctypes.c_uint64, _u8p, _u64p, ctypes.c_uint32,
                                             ctypes.c_uint64, ctypes.c_uint64, _u64pp, _u64pp]
        lib.rko_search_recompute.restype = ctypes.c_int
        lib.rko_brute.argtypes = [_u8p, ctypes.c_uint64, _u8p, _u64p, ctypes.c_uint32,
                                  _u64pp, _u64pp]
        lib.rko_brute.restype = ctypes.c_int
        lib.rko_free.argtypes = [ctypes.c_void_p]
        lib.rko_free.restype = None
        _lib = lib
    return _lib


def _as_u8(a) -> np.ndarray:
    if isinstance(a, (bytes, bytearray, memoryview)):
        a = np.frombuffer(bytes(a), dtype=np.uint8)
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a


def _ptr_u8(a: np.ndarray):
    if a.size == 0:
        a = np.zeros(1, dtype=np.uint8)
    return a.ctypes.data_as(_u8p), a


def pack_patterns(patterns) -> tuple[np.ndarray, np.ndarray]:
    """Concatenate a list of byte strings; returns (bytes u8, offsets u64 of len k+1)."""
    pats = [bytes(p) for p in patterns]
    offs = np.zeros(len(pats) + 1, dtype=np.uint64)
    if pats:
        offs[1:] = np.cumsum([len(p) for p in pats], dtype=np.uint64)
    blob = np.frombuffer(b"".join(pats), dtype=np.uint8) if pats else np.zeros(0, np.uint8)
    return np.ascontiguousarray(blob), offs


def hash(s, d: int = D_DEFAULT, q: int = Q_DEFAULT) -> int:  # noqa: A001 - paper's name
    s = _as_u8(s)
    p, keep = _ptr_u8(s)
    return int(_load().rko_hash(p, s.size, d, q))


def pow_mod(d: int, e: int, q: int = Q_DEFAULT) -> int:
    return int(_load().rko_pow(d, e, q))


def window_hashes(text, m: int, xs, d: int = D_DEFAULT, q: int = Q_DEFAULT) -> np.ndarray:
    text = _as_u8(text)
    xs = np.ascontiguousarray(xs, dtype=np.uint64)
    out = np.zeros(xs.size, dtype=np.uint64)
    p, keep = _ptr_u8(text)
    xsp = xs if xs.size else np.zeros(1, np.uint64)
    outp = out if out.size else np.zeros(1, np.uint64)
    rc = _load().rko_window_hashes(p, text.size, m, d, q, xsp.ctypes.data_as(_u64p), xs.size,
                                   outp.ctypes.data_as(_u64p))
    if rc != 0:
        raise ValueError("rko_window_hashes: invalid arguments (rc=%d)" % rc)
    return out


def _collect(rc, k, offs_p, pos_p, name):
    lib = _load()
    if rc != 0:
        raise ValueError("%s failed (rc=%d)" % (name, rc))
    offsets = np.ctypeslib.as_array(offs_p, shape=(k + 1,)).copy()
    total = int(offsets[k])
    positions = np.ctypeslib.as_array(pos_p, shape=(max(total, 1),))[:total].copy()
    lib.rko_free(ctypes.cast(offs_p, ctypes.c_void_p))
    lib.rko_free(ctypes.cast(pos_p, ctypes.c_void_p))
    return offsets, positions


def search(text, patterns, d: int = D_DEFAULT, q: int = Q_DEFAULT, threads: int = 1):
    """Rolling Rabin-Karp.  Returns (offsets u64[k+1], positions u64[total])."""
    text = _as_u8(text)
    blob, offs = pack_patterns(patterns)
    k = len(offs) - 1
    tp, keep1 = _ptr_u8(text)
    bp, keep2 = _ptr_u8(blob)
    o_p, p_p = _u64p(), _u64p()
    rc = _load().rko_search(tp, text.size, bp, offs.ctypes.data_as(_u64p), k, d, q, int(threads),
                            ctypes.byref(o_p), ctypes.byref(p_p))
    return _collect(rc, k, o_p, p_p, "rko_search")


def search_recompute(text, patterns, d: int = D_DEFAULT, q: int = Q_DEFAULT):
    """The paper's loop: each window hash recomputed by Horner.  O(n*m)."""
    text = _as_u8(text)
    blob, offs = pack_patterns(patterns)
    k = len(offs) - 1
    tp, keep1 = _ptr_u8(text)
    bp, keep2 = _ptr_u8(blob)
    o_p, p_p = _u64p(), _u64p()
    rc = _load().rko_search_recompute(tp, text.size, bp, offs.ctypes.data_as(_u64p), k, d, q,
                                      ctypes.byref(o_p), ctypes.byref(p_p))
    return _collect(rc, k, o_p, p_p, "rko_search_recompute")


def brute(text, patterns):
    """Byte comparison at every window (the definition of an occurrence)."""
    text = _as_u8(text)
    blob, offs = pack_patterns(patterns)
    k = len(offs) - 1
    tp, keep1 = _ptr_u8(text)
    bp, keep2 = _ptr_u8(blob)
    o_p, p_p = _u64p(), _u64p()
    rc = _load().rko_brute(tp, text.size, bp, offs.ctypes.data_as(_u64p), k,
                           ctypes.byref(o_p), ctypes.byref(p_p))
    return _collect(rc, k, o_p, p_p, "rko_brute")


def split(offsets, positions):
    """Per-pattern list view: [positions[offsets[j]:offsets[j+1]] for j]."""
    return [positions[int(offsets[j]):int(offsets[j + 1])] for j in range(len(offsets) - 1)]
