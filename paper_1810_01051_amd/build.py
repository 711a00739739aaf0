"""Builds librk.so (HIP for gfx950) in-tree with hipcc.

    python paper_1810_01051_amd/build.py

Run it as a script (not ``-m``): importing the package loads librk.so.  The
sources compile in parallel (the scan kernels are split by family so that no
single translation unit dominates), then link into one shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librk.so")
SOURCES = (["rk_%s_exact_%s.hip" % (k, g) for g in ("256x132", "512x68", "256x68", "256x36") for k in ("scan", "list")] +
           ["rk_scan_screen.hip", "rk_device.hip", "rk_paper.hip", "rk_noalloc.hip", "rk_host.cpp", "rk_exec.cpp", "rk_tune.cpp",
            "rk_stream.cpp", "rk_server.cpp"])
ARCH = os.environ.get("RK_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-Wno-unused-value", "-Wno-unused-result",
         # packed fp32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        sys.stderr.write(out + "\n")
        raise RuntimeError("build failed: " + " ".join(cmd))
    return out


def _jobs() -> int:
    n = os.cpu_count() or 1
    try:
        n = min(n, int(os.environ.get("MAX_JOBS", n)))
    except ValueError:
        pass
    return max(1, min(n, 16))


def _stale(src: str, obj: str) -> bool:
    """True if obj is missing or older than src or any header of csrc/ and include/."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")]
    inc = os.path.join(os.path.dirname(HERE), "include")
    deps += [os.path.join(inc, h) for h in os.listdir(inc) if h.endswith(".h")]
    return any(os.path.getmtime(d) > t for d in deps)


def build(verbose: bool = False, only_stale: bool = False) -> str:
    """Compile every source to an object (in parallel), then link librk.so.
    Rebuilds everything unless only_stale (then sources whose object is older
    than the source or a header are recompiled)."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    t0 = time.time()

    def one(src):
        obj = os.path.join(objdir, src + ".o")
        if only_stale and not _stale(src, obj):
            return obj, ""
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = ["hipcc", "--offload-arch=" + ARCH] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        return obj, _run(cmd)

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(one, SOURCES))
    objs = []
    for obj, msg in results:
        if verbose and msg.strip():
            print(msg)
        objs.append(obj)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1fs" % (LIB, time.time() - t0))
    return LIB


if __name__ == "__main__":
    build(verbose=True, only_stale="--stale" in sys.argv[1:])
