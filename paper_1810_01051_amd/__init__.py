"""MI355X (gfx950) multi-pattern Rabin-Karp search behind a C ABI (librk.so).

Shah & Oza, "Improved Parallel Rabin-Karp Algorithm Using CUDA": every text
window gets a polynomial hash that is tested against the pattern-hash set and
confirmed byte by byte.  Importing this package loads librk.so; there is no
CPU fallback.
"""
from ._lib import load as _load

_load()

from .search import (BatchPlan, Context, Plan, default_context, search, split)  # noqa: E402,F401
from .server import Server  # noqa: E402,F401

__all__ = ["Context", "Plan", "BatchPlan", "Server", "search", "split", "default_context"]
