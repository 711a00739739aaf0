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


# the sources that decide what the scan kernels read and write: the kernels,
# their descriptors, the table images and the launch geometry
KERNEL_SOURCES = ("rk_scan.h", "rk_dev.h", "rk_exec.cpp", "rk_host.cpp", "rk_internal.h", "rk_runtime.h")


def source_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1810_01051_amd", "csrc")
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def host_cpu():
    """The host's CPU as the bench sees it: logical CPUs of the machine, CPUs
    this process may run on, the thread count the oracle legs use (this
    process's share, at most 16 per GPU) and the lscpu model name."""
    total = os.cpu_count() or 1
    try:
        usable = len(os.sched_getaffinity(0))
    except Exception:
        usable = total
    model = "unknown"
    try:
        import subprocess
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.strip().startswith("Model name"):
                model = line.split(":", 1)[1].strip()
                break
    except Exception:
        pass
    if model == "unknown":
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except Exception:
            pass
    return {"cores_total": total, "cores_usable": usable, "threads": max(1, min(usable, 16)), "cpu_model": model}


def oracle_rate(text_np, patterns, threads: int, target_s: float):
    """The oracle on the first bytes of text_np, sized for about target_s
    seconds: (bytes, seconds, hits)."""
    import oracle
    probe = min(len(text_np), 1 << 24)
    t0 = time.perf_counter()
    oracle.search(text_np[:probe], patterns, threads=threads)
    rate = probe / max(time.perf_counter() - t0, 1e-3)
    sample = int(min(len(text_np), max(probe, rate * target_s)))
    t0 = time.perf_counter()
    off, _ = oracle.search(text_np[:sample], patterns, threads=threads)
    return sample, time.perf_counter() - t0, int(off[-1])


def cpu_baseline(text_np, pattern: bytes, target_s: float = 8.0):
    """The oracle as it stands, timed on the host's cores on the first bytes of
    the same text: one thread, and every usable core (threaded oracle: text
    chunks with an (m-1)-byte overlap), each sized for about target_s seconds."""
    h = host_cpu()
    b1, t1, _ = oracle_rate(text_np, [pattern], 1, target_s)
    bn, tn, hits = oracle_rate(text_np, [pattern], h["threads"], target_s)
    return {"value": round(bn / tn / 1e9, 4), "unit": "GB/s", "cores": h["threads"], "kind": "oracle",
            "sample": "first %d bytes of the same text on %d threads (%.1f s, %d hits); first %d bytes on 1 thread "
                      "(%.1f s)" % (bn, h["threads"], tn, hits, b1, t1),
            "value_1core": round(b1 / t1 / 1e9, 4), **h}


def run_mode(rk, ctx, text, patterns, mode, steps, warmup):
    import torch
    from paper_1810_01051_amd import _lib
    plan = rk.Plan(ctx, patterns, mode)
    n = text.numel()
    scratch = plan.scratch(n, text.device)
    total = plan.count(text, scratch)
    offsets = torch.empty(len(patterns) + 1, dtype=torch.int64, device=text.device)
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
           "positions": positions[:t].clone(), "offsets": offsets.clone(), "cfg": plan_cfg(ctx, mode)}
    plan.close()
    return res


def make_ctx(rk, args):
    """Context with the tuning table and any forced geometry / grid."""
    from paper_1810_01051_amd import _lib
    ctx = rk.Context(0)
    if args.tune and os.path.exists(args.tune):
        ctx.autotune_load(args.tune)
    if args.cfg >= 0:
        ctx.set_option(_lib.RK_OPT_TILE_CFG, args.cfg)
    if args.grid > 0:
        ctx.set_option(_lib.RK_OPT_GRID, args.grid)
    return ctx


def stream_read_ceiling(ctx, text, grids=(256, 512, 1024, 2048, 8192, 32768)):
    """Read bandwidth of the plain streaming kernel (rk_stream_read: every
    16-byte block of the text read once, no compute) over the same buffer,
    best of several grid sizes: the practical HBM read ceiling the scan is
    compared with."""
    import ctypes
    import torch
    from paper_1810_01051_amd import _lib
    n = text.numel() & ~15
    best = 0.0
    for grid in grids:
        out = torch.empty(grid, dtype=torch.int32, device=text.device)
        for _ in range(2):
            ctx.lib.rk_stream_read(ctx.h, ctypes.c_void_p(text.data_ptr()), n, ctypes.c_void_p(out.data_ptr()), grid,
                                   None)
        torch.cuda.synchronize()
        ctx.set_option(_lib.RK_OPT_PROFILE, 1)
        ctx.profile_reset()
        for _ in range(5):
            ctx.lib.rk_stream_read(ctx.h, ctypes.c_void_p(text.data_ptr()), n, ctypes.c_void_p(out.data_ptr()), grid,
                                   None)
        k, ms = ctx.profile(4)
        ctx.set_option(_lib.RK_OPT_PROFILE, 0)
        ctx.profile_reset()
        best = max(best, n / (ms / k / 1e3) / 1e9)
    return round(best, 1)


def plan_cfg(ctx, mode):
    m = {"screen": 2, "exact": 1}[mode]
    return ctx.autotune_choice(m, 32)


# ---------------------------------------------------------------- config 1
def bench_config1(args):
    """1 MiB of i.i.d. a..z text, one m=8 pattern copied from the text and
    planted 100 more times: the latency case (the text sits in the caches, so
    the figure is the time of one whole search, not an HBM fraction).  Every
    search is count (with its total readback) + collect, timed on the host
    around a synchronised call; the oracle checks the result and is timed on
    one host thread and on the threaded path."""
    import numpy as np
    import torch
    import oracle
    import rkgen
    import paper_1810_01051_amd as rk

    s = rkgen.config1()
    text = torch.from_numpy(s.text).to("cuda:0")
    n = s.text.size
    ctx = make_ctx(rk, args)
    runs = max(200, 10 * args.steps)
    out = {}
    # cpu_baseline leg: the oracle timed on one host thread and threaded; its
    # result is also the reference the GPU result is checked against
    cpu = {}
    ref = None
    hc = host_cpu()
    for threads in (1, hc["threads"]):
        ts = []
        for _ in range(5):
            t0 = time.perf_counter()
            ref = oracle.search(s.text, s.patterns, threads=threads)
            ts.append(time.perf_counter() - t0)
        cpu["threads_%d_ms" % threads] = round(float(np.median(ts)) * 1e3, 3)
    for mode in ("screen", "exact"):
        plan = rk.Plan(ctx, s.patterns, mode)
        scratch = plan.scratch(n, text.device)
        total = plan.count(text, scratch)
        offsets = torch.empty(2, dtype=torch.int64, device=text.device)
        positions = torch.empty(max(total, 1), dtype=torch.int64, device=text.device)
        for _ in range(20):
            t = plan.count(text, scratch)
            plan.collect(text, t, scratch, out=(offsets, positions))
        torch.cuda.synchronize()
        lat = []
        for _ in range(runs):
            t0 = time.perf_counter()
            t = plan.count(text, scratch)
            plan.collect(text, t, scratch, out=(offsets, positions))
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
        ok = (offsets.cpu().numpy().astype(np.uint64).tolist() == ref[0].tolist() and
              positions[:t].cpu().numpy().astype(np.uint64).tolist() == ref[1].tolist())
        ls = np.array(lat) * 1e3
        out[mode] = {"p50_ms": round(float(np.percentile(ls, 50)), 4), "p99_ms": round(float(np.percentile(ls, 99)), 4),
                     "min_ms": round(float(ls.min()), 4), "runs": runs, "hits": int(t), "oracle_ok": bool(ok)}
        plan.close()
        log("config1 %s: %s" % (mode, out[mode]))
    line = {
        "metric": "latency of one whole search (count + total readback + collect)",
        "value": out["screen"]["p50_ms"], "unit": "ms", "n_gpus": 1, "steps": runs, "warmup": 20,
        "ms_per_step": out["screen"]["p50_ms"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "single short pattern: %d B i.i.d. a..z text, m=8, 100 planted" % n,
                   "results": out},
        "cpu_baseline": {"unit": "ms", "kind": "oracle", "sample": "the whole workload", "cores": hc["threads"],
                         **cpu, **hc},
    }
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- config 3
def bench_config3(args):
    """1,024 patterns of m=16 (512 sampled, 512 random) over 1 GiB of Zipf
    word text: multi-pattern scan throughput in both modes; the result of the
    first 64 MiB is checked against the oracle."""
    import numpy as np
    import torch
    import rkgen
    import oracle
    import paper_1810_01051_amd as rk
    t0 = time.perf_counter()
    s = rkgen.config3()
    log("config3 generated in %.1fs" % (time.perf_counter() - t0))
    if args.patterns3 != "all":
        # the cost split: the sampled half (hits every ~32 bytes) or the
        # random half (almost no hits) alone
        half = len(s.patterns) // 2
        s.patterns = s.patterns[:half] if args.patterns3 == "sampled" else s.patterns[half:]
    text = torch.from_numpy(s.text).to("cuda:0")
    ctx = make_ctx(rk, args)
    n = text.numel()
    out = {}
    for mode in ("screen", "exact"):
        r = run_mode(rk, ctx, text, s.patterns, mode, args.steps, args.warmup)
        out[mode] = {"GB/s": round(n / (r["ms_per_step"] / 1e3) / 1e9, 2),
                     "scan_GB/s": round(n / (r["scan_ms"] / 1e3) / 1e9, 1),
                     "ms_per_step": round(r["ms_per_step"], 3), "hits": r["total"], "tile_cfg": r["cfg"]}
        log("config3 %s: %s" % (mode, out[mode]))
        if mode == "screen":
            first = r
    # cpu_baseline leg: the oracle timed on the first 64 MiB; its result also
    # checks the GPU result there (windows wholly inside the prefix)
    pre = 64 << 20
    hc = host_cpu()
    threads = hc["threads"]
    t0 = time.perf_counter()
    ro, rp = oracle.search(s.text[:pre], s.patterns, threads=threads)
    dt = time.perf_counter() - t0
    b1, t1, _ = oracle_rate(s.text, s.patterns, 1, 6.0)
    cpu = {"value": round(pre / dt / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": "first 64 MiB of the same text on %d threads (%.1f s); first %d bytes on 1 thread (%.1f s)"
                     % (threads, dt, b1, t1), "value_1core": round(b1 / t1 / 1e9, 4), **hc}
    go = first["offsets"].cpu().numpy().astype(np.int64)
    gp = first["positions"].cpu().numpy().astype(np.int64)
    ok = True
    for j in range(len(s.patterns)):
        a = gp[go[j]:go[j + 1]]
        a = a[a + 16 <= pre]
        b = rp[ro[j]:ro[j + 1]].astype(np.int64)
        if not np.array_equal(a, b):
            ok = False
            break
    line = {
        "metric": "GB/s text scanned (fraction of HBM peak); batched/served p50/p99 latency",
        "value": out["screen"]["GB/s"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": out["screen"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "multi-pattern: %d B Zipf(1.1) word text, %d patterns m=16 (%s of 512 sampled + "
                               "512 random)" % (n, len(s.patterns), args.patterns3),
                   "results": out, "oracle_prefix_64MiB_ok": ok},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- config 4
def bench_config4(args):
    """4,096 uneven searches: one persistent launch over all of them (the batch
    plan's work queue) against one count+collect per instance."""
    import numpy as np
    import torch
    import oracle
    import rkgen
    import paper_1810_01051_amd as rk
    t0 = time.perf_counter()
    insts = rkgen.config4(count=args.count4)
    total_bytes = sum(len(s.text) for s in insts)
    log("config4: %d instances, %d bytes, generated in %.1fs" % (len(insts), total_bytes, time.perf_counter() - t0))
    offs, o = [], 0
    for s in insts:
        offs.append(o)
        o += (len(s.text) + 255) // 256 * 256
    buf = torch.empty(o, dtype=torch.uint8, device="cuda:0")
    for s, off in zip(insts, offs):
        buf[off:off + len(s.text)].copy_(torch.from_numpy(s.text))
    texts = [buf[off:off + len(s.text)] for s, off in zip(insts, offs)]
    torch.cuda.synchronize()
    ctx = make_ctx(rk, args)
    # cpu_baseline leg: the oracle timed on a sample of the instances (every
    # len/12-th); its results also check the batched results of both modes
    sample = list(range(0, len(insts), max(1, len(insts) // 12)))
    hc = host_cpu()
    threads = hc["threads"]
    t0 = time.perf_counter()
    refs = {}
    for i in sample:
        ro, rp = oracle.search(insts[i].text, insts[i].patterns, threads=threads)
        refs[i] = oracle.split(ro, rp)
    dt = time.perf_counter() - t0
    sample_bytes = sum(len(insts[i].text) for i in sample)
    cpu = {"value": round(sample_bytes / dt / 1e9, 4), "unit": "GB/s", "cores": threads, "kind": "oracle",
           "sample": "%d of the %d instances, %d bytes, threaded oracle per instance (%.1f s)"
                     % (len(sample), len(insts), sample_bytes, dt), **hc}
    res = {}
    for mode in ("screen", "exact") if not args.no_exact else ("screen",):
        bp = rk.BatchPlan(ctx, texts, [s.patterns for s in insts], mode)
        for _ in range(args.warmup):
            bp.search()
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            t1 = time.perf_counter()
            off_b, pos_b = bp.search()
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t1)
        el = time.perf_counter() - t0
        batched = {"GB/s": round(total_bytes * args.steps / el / 1e9, 2), "ms_per_batch": round(el * 1e3 / args.steps, 3),
                   "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3),
                   "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3), "hits": int(pos_b.numel())}
        per = bp.split(off_b, pos_b)
        # one launch per instance (plans built outside the timed region)
        plans = [rk.Plan(ctx, s.patterns, mode) for s in insts]
        scratch = [p.scratch(t.numel(), t.device) for p, t in zip(plans, texts)]
        for p, t, sc in zip(plans[:8], texts[:8], scratch[:8]):
            p.collect(t, p.count(t, sc), sc)
        torch.cuda.synchronize()
        done = []
        solo_out = []
        t0 = time.perf_counter()
        for p, t, sc in zip(plans, texts, scratch):
            tot = p.count(t, sc)
            solo_out.append(p.collect(t, tot, sc))
            done.append(time.perf_counter() - t0)
        torch.cuda.synchronize()
        el1 = time.perf_counter() - t0
        svc = np.diff([0.0] + done)
        single = {"GB/s": round(total_bytes / el1 / 1e9, 2), "ms_total": round(el1 * 1e3, 3),
                  "completion_p50_ms": round(float(np.percentile(done, 50)) * 1e3, 3),
                  "completion_p99_ms": round(float(np.percentile(done, 99)) * 1e3, 3),
                  "service_p50_ms": round(float(np.percentile(svc, 50)) * 1e3, 4),
                  "service_p99_ms": round(float(np.percentile(svc, 99)) * 1e3, 4)}
        # parity: batched == solo for every instance, oracle on a sample
        same = True
        for i, (so, sp) in enumerate(solo_out):
            lists = rk.split(so, sp)
            for j in range(len(insts[i].patterns)):
                if not np.array_equal(per[i][j], lists[j]):
                    same = False
        oracle_ok = True
        for i in sample:
            for j in range(len(insts[i].patterns)):
                if per[i][j].astype(np.uint64).tolist() != refs[i][j].tolist():
                    oracle_ok = False
        for p in plans:
            p.close()
        bp.close()
        res[mode] = {"batched": batched, "one_launch_per_instance": single, "batch_equals_solo": same,
                     "oracle_sample_ok": oracle_ok}
        log("config4 %s: %s" % (mode, res[mode]))
    sc = res["screen"]
    line = {
        "metric": "GB/s text scanned (fraction of HBM peak); batched/served p50/p99 latency",
        "value": sc["batched"]["GB/s"], "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sc["batched"]["ms_per_batch"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "batched uneven instances: %d texts log-uniform 4 KiB..16 MiB (%d B total), "
                               "alphabets {4,26,256}, 1..32 patterns m=4..64, half planted" % (len(insts), total_bytes),
                   "instances": len(insts), "text_bytes": total_bytes, "results": res,
                   "speedup_vs_one_launch_per_instance": round(
                       sc["batched"]["GB/s"] / max(sc["one_launch_per_instance"]["GB/s"], 1e-9), 2)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- config 5
def bench_config5(args):
    """Open-loop Poisson request streams against 64 resident corpora served by
    the continuous-batching server; latency submit -> done, throughput."""
    import threading
    import numpy as np
    import torch
    import rkgen
    import paper_1810_01051_amd as rk
    n = args.corpus_bytes
    t0 = time.perf_counter()
    corpora = [rkgen.config5_corpus(i, n) for i in range(args.corpora)]
    torch.cuda.synchronize()
    log("config5: %d corpora x %d bytes in %.1fs" % (len(corpora), n, time.perf_counter() - t0))
    ctx = make_ctx(rk, args)

    def materialise(specs):
        # gather every sampled (offset, length) on the device, one copy back
        idx_c, idx_o, idx_m = [], [], []
        for (_, c, pats) in specs:
            for p in pats:
                if isinstance(p, tuple):
                    idx_c.append(c)
                    idx_o.append(p[0])
                    idx_m.append(p[1])
        got = {}
        if idx_c:
            cs, os_, ms = np.array(idx_c), np.array(idx_o), np.array(idx_m)
            for c in np.unique(cs):
                sel = np.nonzero(cs == c)[0]
                starts = torch.from_numpy(os_[sel]).to("cuda:0")
                lens = torch.from_numpy(ms[sel]).to("cuda:0")
                ends = torch.cumsum(lens, 0)
                tot = int(ends[-1])
                seg = torch.repeat_interleave(torch.arange(len(sel), device="cuda:0"), lens)
                pos = starts[seg] + torch.arange(tot, device="cuda:0") - (ends - lens)[seg]
                blob = corpora[int(c)][pos].cpu().numpy()
                e = ends.cpu().numpy()
                for q, i in enumerate(sel):
                    got[int(i)] = blob[e[q] - ms[i]:e[q]].tobytes()
        out, k = [], 0
        for (t, c, pats) in specs:
            ps = []
            for p in pats:
                if isinstance(p, tuple):
                    ps.append(got[k])
                    k += 1
                else:
                    ps.append(p)
            out.append((t, c, ps))
        return out

    def run(rate, warm, dur, **srv_kw):
        specs = rkgen.config5_request_specs(rate, warm + dur, n, corpora=len(corpora), seed_sub=int(rate))
        reqs = materialise(specs)
        srv = rk.Server(ctx, mode=args.mode, **srv_kw)
        for c in corpora:
            srv.add_corpus(c)
        rids = [None] * len(reqs)
        index = {}
        lat = {}
        stop = threading.Event()

        def releaser():
            # requests complete out of submission order (a step serves every
            # waiting request of its corpus): results are taken from the
            # server's completion queue and released at once, as a serving
            # client consuming them would
            done = 0
            t_last = time.perf_counter()
            while done < len(reqs) and not stop.is_set():
                rid = srv.next_done(timeout=5.0)
                if rid is not None:
                    while rid not in index:  # the submitting thread records it after submit returns
                        time.sleep(0.0001)
                    res = srv.wait(rid, timeout=0.0, fetch=False)
                    lat[index[rid]] = (res["t_done"] - res["t_submit"], res["status"], int(res["offsets"][-1]))
                    srv.release(rid)
                    done += 1
                if time.perf_counter() - t_last > 5:
                    t_last = time.perf_counter()
                    log("config5 rate %g: %d/%d requests done" % (rate, done, len(reqs)))

        th = threading.Thread(target=releaser)
        th.start()
        t_begin = time.perf_counter()
        for i, (t, c, pats) in enumerate(reqs):
            d = t_begin + t - time.perf_counter()
            if d > 0:
                time.sleep(d)
            rids[i] = srv.submit(c, pats)
            index[rids[i]] = i
        t_sub_end = time.perf_counter()
        srv.drain()
        th.join()
        t_end = time.perf_counter()
        st = srv.stats()
        srv.close()
        meas = [i for i, (t, _, _) in enumerate(reqs) if t >= warm]
        ls = np.array([lat[i][0] for i in meas]) * 1e3
        ok = all(lat[i][1] == 0 for i in lat)
        hits = sum(lat[i][2] for i in meas)
        # measured window: from the first measured arrival until the last measured request is done
        tput = len(meas) / max(t_end - (t_begin + warm), 1e-9)
        return {"offered_req_s": rate, "requests": len(meas), "achieved_req_s": round(tput, 1),
                "p50_ms": round(float(np.percentile(ls, 50)), 2), "p99_ms": round(float(np.percentile(ls, 99)), 2),
                "mean_ms": round(float(ls.mean()), 2), "all_ok": bool(ok), "hits": int(hits),
                "steps": st["steps"], "merged_patterns": st["merged_patterns"],
                "request_patterns": st["request_patterns"],
                "scan_GB/s_while_busy": round(st["bytes_scanned"] / max(st["busy_s"], 1e-9) / 1e9, 1),
                "admission_waits": st["admission_waits"], "step_splits": st["step_splits"], "failed": st["failed"],
                "arena_high_water_GiB": round(st["arena_high_water"] / 2**30, 2),
                "submit_lag_s": round(t_sub_end - t_begin - warm - dur, 3)}

    results = {}
    for rate in args.rates:
        results["batched_%d" % rate] = run(rate, args.warm5, args.duration5, arena_bytes=args.arena,
                                           max_inflight=args.inflight, max_step_patterns=args.step_patterns,
                                           use_graphs=True)
        log("config5 batched %d: %s" % (rate, results["batched_%d" % rate]))
    # graphs off with everything else held (merging, steps in flight): what
    # launching each step's passes as graphs is worth
    for rate in ([] if args.no_graph_ab else args.rates):
        results["batched_no_graphs_%d" % rate] = run(rate, args.warm5, args.duration5, arena_bytes=args.arena,
                                                     max_inflight=args.inflight,
                                                     max_step_patterns=args.step_patterns, use_graphs=False)
        log("config5 batched, no graphs %d: %s" % (rate, results["batched_no_graphs_%d" % rate]))
    # the baseline: one request per step, one step at a time, plain launches,
    # on the same request stream at every offered rate
    for rate in ([] if args.no_unbatched else args.rates):
        results["one_request_per_launch_%d" % rate] = run(rate, args.warm5, args.duration5_base or args.duration5,
                                                          arena_bytes=args.arena, max_inflight=1,
                                                          max_step_requests=1, use_graphs=False)
        log("config5 unbatched %d: %s" % (rate, results["one_request_per_launch_%d" % rate]))
    top = results["batched_%d" % max(args.rates)]
    line = {
        "metric": "GB/s text scanned (fraction of HBM peak); batched/served p50/p99 latency",
        "value": top["achieved_req_s"], "unit": "req/s", "n_gpus": 1, "steps": top["steps"], "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "serving: Poisson requests over %d resident corpora of %d B (Zipf word text), "
                               "1..256 patterns m=4..64 per request" % (len(corpora), n),
                   "mode": args.mode, "results": results},
    }
    print(json.dumps(line), flush=True)


# ---------------------------------------------------------------- paper mode
PAPER_TABLE12_MS = {  # Tables 1-2 (320 MB DNA, m = 7): GT 920 and GT 630M milliseconds per threads/block
    32: (4718.75, 10638.17), 64: (2708.375, 5931.667), 128: (1715.79, 3600.603), 256: (1220.096, 2434.065),
    512: (971.2466, 1787.352), 1024: (847.1143, 1495.54)}
PAPER_TABLE3_MS = {25: 7.51616, 50: 13.82605, 100: 26.37414, 200: 51.32698, 800: 201.1771}  # GT 920, file size unstated


def bench_paper(args):
    """The paper's own experiments rerun on MI355X in paper mode (one thread
    per offset, the shift-add hash recomputed over m bytes from device
    memory): a 320e6-byte i.i.d. DNA text, m = 7, threads per block 32..1024
    (Tables 1-2), then m = 25..800 at 1024 threads per block (Table 3) beside
    the tiled scans.  One JSON line per point; the paper's own times are
    context (other GPUs, other file)."""
    import numpy as np
    import torch
    import oracle
    import rkgen
    import paper_1810_01051_amd as rk
    from paper_1810_01051_amd import _lib
    n = args.paper_n
    g = rkgen.rng(80, 0)
    text_np = rkgen.iid_text(g, n, rkgen.ACGT)
    text = torch.from_numpy(text_np).to("cuda:0")
    ctx = make_ctx(rk, args)
    hc = host_cpu()

    def paper_time(pat, tpb, reps):
        flags = ctx.paper_search(text, pat, tpb)
        torch.cuda.synchronize()
        ctx.set_option(_lib.RK_OPT_PROFILE, 1)
        ctx.profile_reset()
        for _ in range(reps):
            ctx.paper_search(text, pat, tpb)
        k, ms = ctx.profile(5)
        ctx.set_option(_lib.RK_OPT_PROFILE, 0)
        ctx.profile_reset()
        return ms / k, flags

    def tiled_time(pat, mode, reps):
        return run_mode(rk, ctx, text, [pat], mode, reps, 2)

    def emit(value_ms, extra, cpu=None):
        line = {"metric": "paper-mode search time (the paper's Tables 1-3)", "value": round(value_ms, 4), "unit": "ms",
                "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": round(value_ms, 4),
                "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
                "data": "synthetic", "config": extra}
        if cpu:
            line["cpu_baseline"] = cpu
        print(json.dumps(line), flush=True)

    # Tables 1-2: m = 7, threads per block 32..1024
    o = int(g.integers(0, n - 7))
    pat7 = text_np[o:o + 7].tobytes()
    ro, rp = oracle.search(text_np, [pat7], threads=hc["threads"])
    # the paper's sequential loop (the oracle's recompute search, one thread) on a bounded prefix
    pre = min(n, 32 << 20)
    t0 = time.perf_counter()
    oracle.search_recompute(text_np[:pre], [pat7], d=2, q=1 << 32)
    dt = time.perf_counter() - t0
    cpu = {"value": round(dt * n / pre * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
           "sample": "the paper's sequential loop (hash recomputed per window, d=2, q=2^32) on the first %d bytes "
                     "in %.2f s, scaled to the whole text" % (pre, dt), **hc}
    for tpb in (32, 64, 128, 256, 512, 1024):
        ms, flags = paper_time(pat7, tpb, args.steps)
        pos = ctx.paper_positions(flags).cpu().numpy().astype(np.uint64)
        ok = pos.tolist() == rp.tolist()
        pt = PAPER_TABLE12_MS[tpb]
        emit(ms, {"workload": "paper mode: %d B i.i.d. ACGT text, m=7, %d threads/block" % (n, tpb),
                  "threads_per_block": tpb, "m": 7, "GB/s": round(n / (ms / 1e3) / 1e9, 2), "hits": int(pos.size),
                  "oracle_ok": ok, "paper_ms_GT920": pt[0], "paper_ms_GT630M": pt[1],
                  "speedup_vs_GT920": round(pt[0] / ms, 1)}, cpu if tpb == 1024 else None)
        log("paper tpb %d: %.3f ms, oracle %s" % (tpb, ms, ok))
    # Table 3: pattern length, paper mode at 1024 threads/block beside the tiled scans
    for m in (25, 50, 100, 200, 800):
        o = int(g.integers(0, n - m))
        pat = text_np[o:o + m].tobytes()
        ms, flags = paper_time(pat, 1024, max(3, args.steps // 2))
        pos = ctx.paper_positions(flags)
        tiled = {}
        for mode in ("screen", "exact"):
            r = tiled_time(pat, mode, max(3, args.steps // 2))
            same = bool(torch.equal(r["positions"], pos))
            tiled[mode] = {"ms_per_step": round(r["ms_per_step"], 4), "scan_ms": round(r["scan_ms"], 4),
                           "GB/s": round(n / (r["ms_per_step"] / 1e3) / 1e9, 1), "same_positions": same}
        emit(ms, {"workload": "paper mode: %d B i.i.d. ACGT text, m=%d, 1024 threads/block" % (n, m),
                  "threads_per_block": 1024, "m": m, "GB/s": round(n / (ms / 1e3) / 1e9, 2),
                  "hits": int(pos.numel()), "paper_ms_GT920_table3": PAPER_TABLE3_MS[m], "tiled_scan": tiled})
        log("paper m %d: %.3f ms, tiled %s" % (m, ms, tiled))


# ---------------------------------------------------------------- streamed
def bench_stream(args):
    """A text in host memory (pageable, args.stream_n bytes of i.i.d. ACGT)
    searched by rk_search_host in pieces of args.piece bytes: link-bound
    end-to-end GB/s (staging, host-to-device copy and search overlapped), with
    the same text resident on the device for comparison.  The result is
    checked against the device-resident search."""
    import numpy as np
    import torch
    import rkgen
    import paper_1810_01051_amd as rk
    n = args.stream_n
    t0 = time.perf_counter()
    s = rkgen.config2(n=n, plants=1000)
    log("stream: %d bytes generated in %.1fs" % (n, time.perf_counter() - t0))
    ctx = make_ctx(rk, args)
    res = {}
    for mode in ("screen", "exact"):
        plan = rk.Plan(ctx, s.patterns, mode)
        plan.search_host(s.text[:1 << 26], args.piece)  # warm-up
        ts = []
        for _ in range(max(1, args.steps // 5)):
            t0 = time.perf_counter()
            off, pos = plan.search_host(s.text, args.piece)
            ts.append(time.perf_counter() - t0)
        el = min(ts)
        text = torch.from_numpy(s.text).to("cuda:0")
        ro, rp = plan.search(text)
        torch.cuda.synchronize()
        same = off.tolist() == ro.cpu().numpy().astype(np.uint64).tolist() and \
            pos.tolist() == rp.cpu().numpy().astype(np.uint64).tolist()
        del text
        torch.cuda.empty_cache()
        plan.close()
        res[mode] = {"GB/s": round(n / el / 1e9, 2), "s": round(el, 3), "hits": int(off[-1]),
                     "same_as_resident": bool(same)}
        log("stream %s: %s" % (mode, res[mode]))
    # host-to-device copy ceiling over the same link (pinned source)
    pin = torch.empty(1 << 30, dtype=torch.uint8, pin_memory=True)
    dst = torch.empty(1 << 30, dtype=torch.uint8, device="cuda:0")
    dst.copy_(pin, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(4):
        dst.copy_(pin, non_blocking=True)
    torch.cuda.synchronize()
    h2d = 4 * (1 << 30) / (time.perf_counter() - t0) / 1e9
    line = {"metric": "GB/s text scanned, streamed from host memory", "value": res["screen"]["GB/s"],
            "unit": "GB/s", "n_gpus": 1, "steps": max(1, args.steps // 5), "warmup": 1,
            "ms_per_step": round(res["screen"]["s"] * 1e3, 1), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u8", "data": "synthetic",
            "config": {"workload": "streamed search: %d B i.i.d. ACGT text in pageable host memory, m=32, "
                                   "pieces of %d B" % (n, args.piece), "results": res,
                       "h2d_copy_GBps_pinned": round(h2d, 1)}}
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 32, help="text bytes (default 4 GiB)")
    ap.add_argument("--mode", default="screen", choices=["screen", "exact"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-exact", action="store_true", help="skip the every-window exact-hash measurement")
    ap.add_argument("--tune", default=os.path.join(ROOT, "paper_1810_01051_amd", "autotune_gfx950.json"))
    ap.add_argument("--cfg", type=int, default=-1, help="force a scan geometry (rk_tile_cfg index)")
    ap.add_argument("--grid", type=int, default=0, help="force the persistent grid size")
    ap.add_argument("--workload", default="config2",
                    choices=["config1", "config2", "config3", "config4", "config5", "paper", "stream"],
                    help="config2 (default): the single-pattern DNA scan; config1: the 1 MiB latency case; config3: "
                         "1,024 patterns over Zipf text; config4: batched uneven instances; config5: serving; "
                         "paper: the paper's Tables 1-3 in paper mode")
    ap.add_argument("--paper-n", type=int, default=320 * 10 ** 6, help="paper workload text bytes")
    ap.add_argument("--stream-n", type=int, default=16 << 30, help="stream workload host text bytes")
    ap.add_argument("--piece", type=int, default=512 << 20, help="stream workload piece bytes")
    ap.add_argument("--count4", type=int, default=4096, help="config4 instances")
    ap.add_argument("--patterns3", default="all", choices=["all", "sampled", "random"],
                    help="config3: every pattern, or only the sampled / only the random half")
    ap.add_argument("--corpora", type=int, default=64, help="config5 corpora")
    ap.add_argument("--corpus-bytes", type=int, default=1 << 30, help="config5 bytes per corpus")
    ap.add_argument("--rates", type=float, nargs="+", default=[500, 2000, 8000], help="config5 offered req/s")
    ap.add_argument("--warm5", type=float, default=1.0)
    ap.add_argument("--duration5", type=float, default=10.0)
    ap.add_argument("--duration5-base", type=float, default=None,
                    help="config5: measured window of the one-request-per-launch baseline (default: --duration5)")
    ap.add_argument("--arena", type=int, default=64 << 30, help="config5 server output arena bytes")
    ap.add_argument("--inflight", type=int, default=2, help="config5 steps in flight")
    ap.add_argument("--step-patterns", type=int, default=None,
                    help="config5 merged patterns per step (default: the library's)")
    ap.add_argument("--no-unbatched", action="store_true", help="config5: skip the one-request-per-launch runs")
    ap.add_argument("--no-graph-ab", action="store_true", help="config5: skip the graphs-off runs")
    ap.add_argument("--calib-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (for PMC byte-counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: a search over several GPUs splits the text into ranges with an "
              "(m-1)-byte halo, each range being a one-GPU search like this one; run with --gpus 1", file=sys.stderr)
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

    if args.workload == "config1":
        return bench_config1(args)
    if args.workload == "config3":
        return bench_config3(args)
    if args.workload == "config4":
        return bench_config4(args)
    if args.workload == "config5":
        return bench_config5(args)
    if args.workload == "paper":
        return bench_paper(args)
    if args.workload == "stream":
        return bench_stream(args)

    import rkgen
    import paper_1810_01051_amd as rk

    t0 = time.perf_counter()
    s = rkgen.config2(n=args.n)
    pattern = s.patterns[0]
    log("generated %d bytes in %.1fs" % (args.n, time.perf_counter() - t0))
    text = torch.from_numpy(s.text).to("cuda:0")
    torch.cuda.synchronize()
    ctx = make_ctx(rk, args)

    res = run_mode(rk, ctx, text, [pattern], args.mode, args.steps, args.warmup)
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
        "roofline": {"bound": "hbm", "kernel": "scan of the rk_count pass (single-bucket scan_list_kernel, "
                                               "geometry %d)" % res["cfg"],
                     "achieved": round(scan_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(scan_gbs / HBM_PEAK_GBS, 4),
                     "traffic": traffic["bytes_per_launch"] if traffic else None,
                     "avg_launch_ms": round(res["scan_ms"], 4)},
    }
    if not args.no_exact:
        other = "exact" if args.mode == "screen" else "screen"
        r2 = run_mode(rk, ctx, text, [pattern], other, max(3, args.steps // 2), 1)
        line["config"]["%s_mode" % other] = {
            "GB/s": round(n / (r2["ms_per_step"] / 1e3) / 1e9, 2),
            "scan_GB/s": round(n / (r2["scan_ms"] / 1e3) / 1e9, 1),
            "scan_frac": round(n / (r2["scan_ms"] / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            "hits": r2["total"],
            "same_positions": bool(torch.equal(r2["positions"], res["positions"]))}
        log("%s: %.3f ms/step, scan %.3f ms" % (other, r2["ms_per_step"], r2["scan_ms"]))
    sr = stream_read_ceiling(ctx, text)
    line["roofline"]["stream_read_GBps"] = sr
    line["roofline"]["frac_of_stream_read"] = round(scan_gbs / sr, 4)
    log("stream-read ceiling %.1f GB/s" % sr)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(s.text, pattern)
        log("cpu baseline %s" % line["cpu_baseline"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
