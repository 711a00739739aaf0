"""Host-only checks of the C ABI: librk.so loads and exports every function
that include/rk.h declares; pure host calls answer without a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("rk.h", "rk_server.h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(rk_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("rk_ctx_create", "rk_plan_create", "rk_count", "rk_collect", "rk_window_hashes", "rk_scan_dump",
              "rk_batch_plan_create", "rk_autotune", "rk_server_create", "rk_server_submit", "rk_server_poll"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1810_01051_amd import _lib
    lib = _lib.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # every declared function has a ctypes signature in the binding
    assert not [n for n in declared_functions() if n not in _lib.SIGNATURES]


def test_host_only_calls():
    from paper_1810_01051_amd import _lib
    lib = _lib.load()
    assert lib.rk_status_string(_lib.RK_ENOSPACE) == b"RK_ENOSPACE"
    assert lib.rk_tile_cfg_count() >= 1
    wg, c, t = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    for i in range(lib.rk_tile_cfg_count()):
        assert lib.rk_tile_cfg(i, ctypes.byref(wg), ctypes.byref(c), ctypes.byref(t)) == 0
        assert wg.value % 64 == 0 and t.value == wg.value * c.value and t.value % 16 == 0
        # windows per thread = 4 * odd keeps the per-thread LDS dword reads conflict-free
        assert c.value % 4 == 0 and (c.value // 4) % 2 == 1
    assert lib.rk_tile_cfg(99, None, None, None) == _lib.RK_EINVAL
    # null arguments are rejected without touching a device
    assert lib.rk_ctx_create(0, 256, (1 << 61) - 1, None) == _lib.RK_EINVAL
    assert lib.rk_ctx_create(0, 10, (1 << 61) - 1, ctypes.byref(ctypes.c_void_p())) == _lib.RK_EUNSUPPORTED


def test_host_hash_matches_closed_form():
    """rk_hash (the library's own host arithmetic) against the big-endian closed form."""
    from paper_1810_01051_amd import _lib
    import numpy as np
    lib = _lib.load()
    rng = np.random.default_rng(5)
    for m in [1, 2, 7, 8, 9, 31, 32, 33, 64, 200]:
        w = rng.integers(0, 256, size=m, dtype=np.uint8)
        out = ctypes.c_uint64()
        assert lib.rk_hash(None, w.ctypes.data_as(ctypes.c_void_p), m, ctypes.byref(out)) == 0
        assert out.value == int.from_bytes(w.tobytes(), "big") % ((1 << 61) - 1)


def test_python_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1810_01051_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(ImportError):
        _lib.load()
