"""Builds librk.so (HIP for gfx950) in-tree with hipcc.

    python paper_1810_01051_amd/build.py

Run it as a script (not ``-m``): importing the package loads librk.so.  The
sources compile in parallel (the scan kernels are split by family so that no
single translation unit dominates), then link into one shared library.
"""
from __future__ import annotations

import json
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


def _resource_usage(out: str) -> dict:
    """Per-kernel resource usage from the compiler's kernel-resource-usage
    remarks: VGPRs, SGPRs, scratch bytes per lane, dynamic stack, occupancy."""
    kernels, cur = {}, None
    for line in out.splitlines():
        if "kernel-resource-usage" not in line:
            continue
        body = line.split("remark:", 1)[-1].split("[-Rpass", 1)[0].strip()
        key, _, val = body.partition(":")
        key, val = key.strip(), val.strip()
        if key == "Function Name":
            cur = kernels.setdefault(val, {})
        elif cur is not None:
            if key == "VGPRs":
                cur["vgprs"] = int(val)
            elif key == "TotalSGPRs":
                cur["sgprs"] = int(val)
            elif key.startswith("ScratchSize"):
                cur["scratch"] = int(val)
            elif key == "Dynamic Stack":
                cur["dyn_stack"] = val.lower() == "true"
            elif key.startswith("Occupancy"):
                cur["occupancy"] = int(val)
            elif key.startswith("LDS Size"):
                cur["lds"] = int(val)
            elif key == "VGPRs Spill":
                cur["vgpr_spill"] = int(val)
            elif key == "SGPRs Spill":
                cur["sgpr_spill"] = int(val)
    return kernels


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
        usage = obj + ".usage.json"
        if only_stale and not _stale(src, obj) and os.path.exists(usage):
            return obj, "", json.load(open(usage))
        hip = src.endswith(".hip")
        lang = ["-x", "hip", "-Rpass-analysis=kernel-resource-usage"] if hip else []
        cmd = ["hipcc", "--offload-arch=" + ARCH] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        out = _run(cmd)
        kernels = _resource_usage(out) if hip else {}
        json.dump(kernels, open(usage, "w"), indent=1, sort_keys=True)
        msg = "\n".join(l for l in out.splitlines() if "kernel-resource-usage" not in l)
        return obj, msg, kernels

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(one, SOURCES))
    objs, kernels = [], {}
    for obj, msg, k in results:
        if verbose and msg.strip():
            print(msg)
        objs.append(obj)
        kernels.update(k)
    json.dump(kernels, open(os.path.join(objdir, "resource_usage.json"), "w"), indent=1, sort_keys=True)
    # no kernel may keep anything on a per-lane stack (a called, outlined
    # function or a spilled array): the scans read LDS through addresses
    # they form themselves and must stay one straight-line kernel
    stack = sorted(k for k, v in kernels.items() if v.get("scratch", 0) or v.get("dyn_stack") or v.get("vgpr_spill", 0))
    if stack:
        raise RuntimeError("kernels with a private-segment stack: " + ", ".join(stack))
    tmp = LIB + ".tmp%d" % os.getpid()
    _run(["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1fs" % (LIB, time.time() - t0))
    return LIB


if __name__ == "__main__":
    build(verbose=True, only_stale="--stale" in sys.argv[1:])
