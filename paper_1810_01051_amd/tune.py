"""Regenerates the scan-geometry table of this GPU (rk_autotune) and writes it
as JSON; the package's table for gfx950 is autotune_gfx950.json next to this
file.

    python -m paper_1810_01051_amd.tune [--n BYTES] [--lengths 4 8 16 32 64] [--out PATH]
"""
from __future__ import annotations

import argparse
import os

from .search import Context


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--n", type=int, default=1 << 31, help="synthetic text bytes for the one-pattern timings")
    ap.add_argument("--lengths", type=int, nargs="+", default=[4, 8, 16, 32, 64])
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_gfx950.json"))
    ap.add_argument("--device", type=int, default=0)
    a = ap.parse_args()
    ctx = Context(a.device)
    ctx.autotune(a.n, a.lengths, a.out)
    ctx.close()
    print("wrote %s" % a.out)


if __name__ == "__main__":
    main()
