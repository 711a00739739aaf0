"""Builds librk.so (HIP for gfx950) in-tree with hipcc.

    python paper_1810_01051_amd/build.py [--out PATH] [-D NAME=VALUE ...]

Run it as a script (not ``-m``): importing the package loads librk.so.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librk.so")
SOURCES = ["rk_device.hip", "rk_host.cpp", "rk_exec.cpp", "rk_tune.cpp", "rk_server.cpp"]
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


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every source to an object, then link librk.so (always rebuilds).
    ``defines`` (e.g. ["RK_PREFETCH=0"]) select build variants of the scan."""
    objdir = os.path.join(HERE, "_build" if out == LIB else "_build_" + os.path.basename(out).replace(".", "_"))
    os.makedirs(objdir, exist_ok=True)
    objs = []
    t0 = time.time()
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = (["hipcc", "--offload-arch=" + ARCH] + FLAGS + ["-D" + d for d in defines] + lang +
               ["-c", os.path.join(CSRC, src), "-o", obj])
        msg = _run(cmd)
        if verbose and msg.strip():
            print(msg)
        objs.append(obj)
    tmp = out + ".tmp%d" % os.getpid()
    _run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, out)
    if verbose:
        print("built %s in %.1fs" % (out, time.time() - t0))
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=LIB)
    ap.add_argument("-D", dest="defines", action="append", default=[])
    a = ap.parse_args()
    build(verbose=True, out=a.out, defines=a.defines)
