#!/usr/bin/env python3
"""Benchmark of the Rabin-Karp hot path on one MI355X.

Workload (the single-pattern DNA search of the paper's experiments, Sec. 4,
scaled to one GPU's share): 4 GiB of i.i.d. {A,C,G,T} text, one random ACGT
pattern of length 32 planted at 10,000 non-overlapping seeded offsets.  A step
is the whole search: rk_count (one pass over the text: window hashes, set
test, byte verification, per-tile hit staging) plus rk_collect (tile-count
scan, compaction into the sorted position list).  The text is resident in HBM
before timing starts.

Prints one JSON line: GB/s of text scanned, the scan kernel's HBM roofline
fraction (HIP events on the library's launch stream) and the CPU oracle's
throughput on the machine's host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def load_traffic(kernel_tag: str):
    """HBM bytes per launch measured with rocprofv3 PMC counters, if a profile
    for the current kernel sources is committed (profiles/traffic.json)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except Exception:
        return None
    e = d.get(kernel_tag)
    if not e or e.get("source_sha") != source_sha():
        return None
    return e


def source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1810_01051_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def cpu_baseline(text_np, pattern: bytes, target_s: float = 10.0):
    """The oracle as it stands, on the first bytes of the same text, sized for
    about target_s seconds of work."""
    import oracle
    threads = max(1, min(os.cpu_count() or 1, 16))
    probe = min(len(text_np), 1 << 25)
    t0 = time.perf_counter()
    oracle.search(text_np[:probe], [pattern], threads=threads)
    dt = max(time.perf_counter() - t0, 1e-3)
    rate = probe / dt
    sample = int(min(len(text_np), max(probe, rate * target_s)))
    t0 = time.perf_counter()
    off, pos = oracle.search(text_np[:sample], [pattern], threads=threads)
    dt = time.perf_counter() - t0
    return {"value": round(sample / dt / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": "first %d bytes of the same text (%.1f s, %d hits)" % (sample, dt, int(off[-1])),
            "cpu_model": cpu_model()}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def run_mode(rk, ctx, text, pattern, mode, steps, warmup):
    import torch
    from paper_1810_01051_amd import _lib
    plan = rk.Plan(ctx, [pattern], mode)
    n = text.numel()
    scratch = plan.scratch(n, text.device)
    total = plan.count(text, scratch)
    offsets = torch.empty(2, dtype=torch.int64, device=text.device)
    positions = torch.empty(max(total, 1), dtype=torch.int64, device=text.device)
    for _ in range(warmup):
        t = plan.count(text, scratch)
        plan.collect(text, t, scratch, out=(offsets, positions))
    torch.cuda.synchronize()
    ctx.set_option(_lib.RK_OPT_PROFILE, 1)
    ctx.profile_reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        t = plan.count(text, scratch)
        plan.collect(text, t, scratch, out=(offsets, positions))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    launches, scan_ms = ctx.profile(0)
    _, all_ms = ctx.profile(3)
    ctx.set_option(_lib.RK_OPT_PROFILE, 0)
    ctx.profile_reset()
    res = {"total": int(t), "ms_per_step": elapsed * 1e3 / steps, "scan_launches": launches,
           "scan_ms": scan_ms / max(launches, 1), "device_ms_per_step": all_ms / steps,
           "positions": positions[:t].clone(), "cfg": plan_cfg(ctx, mode)}
    plan.close()
    return res


def plan_cfg(ctx, mode):
    m = {"screen": 2, "exact": 1}[mode]
    return ctx.autotune_choice(m, 32)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 32, help="text bytes (default 4 GiB)")
    ap.add_argument("--mode", default="screen", choices=["screen", "exact"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-exact", action="store_true", help="skip the every-window exact-hash measurement")
    ap.add_argument("--tune", default=os.path.join(ROOT, "profiles", "autotune_gfx950.json"))
    ap.add_argument("--cfg", type=int, default=-1, help="force a scan geometry (rk_tile_cfg index)")
    ap.add_argument("--grid", type=int, default=0, help="force the persistent grid size")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (for PMC byte-counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build measures one GPU only (the search shards by text range with an "
              "(m-1)-byte halo; see DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calib_copy:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
        b = torch.empty_like(a)
        a.fill_(7)
        torch.cuda.synchronize()
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": 1 << 30, "launches": 3}))
        return

    import rkgen
    import paper_1810_01051_amd as rk

    t0 = time.perf_counter()
    s = rkgen.config2(n=args.n)
    pattern = s.patterns[0]
    log("generated %d bytes in %.1fs" % (args.n, time.perf_counter() - t0))
    text = torch.from_numpy(s.text).to("cuda:0")
    torch.cuda.synchronize()
    ctx = rk.Context(0)
    if args.tune and os.path.exists(args.tune):
        ctx.autotune_load(args.tune)
    from paper_1810_01051_amd import _lib
    if args.cfg >= 0:
        ctx.set_option(_lib.RK_OPT_TILE_CFG, args.cfg)
    if args.grid > 0:
        ctx.set_option(_lib.RK_OPT_GRID, args.grid)

    res = run_mode(rk, ctx, text, pattern, args.mode, args.steps, args.warmup)
    log("%s: %.3f ms/step, scan %.3f ms" % (args.mode, res["ms_per_step"], res["scan_ms"]))
    # result check: every plant found, list ascending, each position byte-matches
    pos = res["positions"].cpu().numpy()
    plants = s.manifest["plants"]
    ok = (np.all(np.diff(pos) > 0) and set(plants.tolist()) <= set(pos.tolist()) and
          all(s.text[x:x + len(pattern)].tobytes() == pattern for x in pos[:2000].tolist()))
    n = args.n
    gbs = n / (res["ms_per_step"] / 1e3) / 1e9
    scan_gbs = n / (res["scan_ms"] / 1e3) / 1e9
    traffic = load_traffic("scan_%s" % args.mode)
    line = {
        "metric": "GB/s text scanned (fraction of HBM peak); batched/served p50/p99 latency",
        "value": round(gbs, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "single pattern over DNA: %d B i.i.d. ACGT text, m=32, 10000 planted" % n,
                   "n": n, "m": 32, "k": 1, "mode": args.mode, "tile_cfg": res["cfg"],
                   "hits": res["total"], "result_check": bool(ok)},
        "roofline": {"bound": "hbm", "kernel": "scan_kernel (rk_count pass)",
                     "achieved": round(scan_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(scan_gbs / HBM_PEAK_GBS, 4),
                     "traffic": traffic["bytes_per_launch"] if traffic else None,
                     "avg_launch_ms": round(res["scan_ms"], 4)},
    }
    if not args.no_exact:
        other = "exact" if args.mode == "screen" else "screen"
        r2 = run_mode(rk, ctx, text, pattern, other, max(3, args.steps // 2), 1)
        line["config"]["%s_mode" % other] = {
            "GB/s": round(n / (r2["ms_per_step"] / 1e3) / 1e9, 2),
            "scan_GB/s": round(n / (r2["scan_ms"] / 1e3) / 1e9, 1),
            "scan_frac": round(n / (r2["scan_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "hits": r2["total"],
            "same_positions": bool(torch.equal(r2["positions"], res["positions"]))}
        log("%s: %.3f ms/step, scan %.3f ms" % (other, r2["ms_per_step"], r2["scan_ms"]))
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(s.text, pattern)
        log("cpu baseline %s" % line["cpu_baseline"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
