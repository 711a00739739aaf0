"""GPU parity: librk (through its C ABI) against the CPU oracle, element by
element, on seeded inputs.  Integer results, so the bar is exact equality."""
import ctypes
import os

import numpy as np
import pytest

import oracle
import rkgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

Q = (1 << 61) - 1
MODES = ["screen", "exact"]


@pytest.fixture(scope="module")
def rk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1810_01051_amd as rk
    return rk


@pytest.fixture(scope="module")
def ctx(rk):
    c = rk.Context(0)
    yield c
    c.close()


def dev(a):
    if isinstance(a, (bytes, bytearray)):
        a = np.frombuffer(bytes(a), dtype=np.uint8)
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint8).copy()).to("cuda:0")
    if t.numel() == 0:
        t = torch.empty(0, dtype=torch.uint8, device="cuda:0")
    return t


def run(ctx, rk, text_np, pats, mode, opts=None):
    opts = opts or {}
    text = dev(text_np)
    for k, v in opts.items():
        ctx.set_option(k, v)
    try:
        plan = rk.Plan(ctx, pats, mode)
        off, pos = plan.search(text)
        torch.cuda.synchronize()
        plan.close()
    finally:
        for k in opts:
            ctx.set_option(k, {1: 0, 2: -1, 3: 0, 4: 0, 5: -1}[k])
    return off.cpu().numpy().astype(np.uint64), pos.cpu().numpy().astype(np.uint64)


def assert_same(got, ref, label=""):
    go, gp = got
    ro, rp = ref
    assert np.array_equal(go, ro), "offsets differ %s" % label
    if not np.array_equal(gp, rp):
        lists_g = oracle.split(go, gp)
        lists_r = oracle.split(ro, rp)
        for j, (a, b) in enumerate(zip(lists_g, lists_r)):
            if a.tolist() != b.tolist():
                extra = sorted(set(a.tolist()) - set(b.tolist()))[:5]
                miss = sorted(set(b.tolist()) - set(a.tolist()))[:5]
                raise AssertionError("pattern %d differs %s: extra %s missing %s" % (j, label, extra, miss))
        raise AssertionError("positions differ %s" % label)


@pytest.mark.parametrize("mode", MODES)
def test_config1_full(ctx, rk, mode):
    s = rkgen.config1()
    got = run(ctx, rk, s.text, s.patterns, mode)
    ref = oracle.search(s.text, s.patterns)
    assert int(ref[0][-1]) == 101
    assert_same(got, ref, "config1 " + mode)


@pytest.mark.parametrize("mode", MODES)
def test_config2_reduced(ctx, rk, mode):
    s = rkgen.config2(n=(1 << 23) + 77, plants=300)
    got = run(ctx, rk, s.text, s.patterns, mode)
    ref = oracle.search(s.text, s.patterns, threads=4)
    assert int(ref[0][-1]) == 300
    assert_same(got, ref, "config2 " + mode)


TUNE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1810_01051_amd",
                    "autotune_gfx950.json")
THREADS = min(os.cpu_count() or 1, 16)


@pytest.fixture(scope="module")
def bench_ctx(rk):
    """A context in the launch configuration bench.py times (its tuning table)."""
    c = rk.Context(0)
    if os.path.exists(TUNE):
        c.autotune_load(TUNE)
    yield c
    c.close()


@pytest.fixture(scope="module")
def config2_full():
    return rkgen.config2()


@pytest.mark.parametrize("mode", MODES)
def test_config2_full_size(bench_ctx, rk, config2_full, mode):
    """Config 2 at its full size (4 GiB, m=32, 10,000 plants), element by
    element against the threaded oracle, plus the window hashes of sampled
    windows against the oracle's direct evaluation."""
    s = config2_full
    got = run(bench_ctx, rk, s.text, s.patterns, mode)
    ref = oracle.search(s.text, s.patterns, threads=THREADS)
    assert int(ref[0][-1]) == 10000
    assert_same(got, ref, "config2 full " + mode)
    if mode == "exact":
        g = rkgen.rng(2, 99)
        xs = np.concatenate([g.integers(0, s.text.size - 32, size=2000), s.manifest["plants"][:500]])
        text = dev(s.text)
        gh = bench_ctx.window_hashes(text, 32, torch.from_numpy(xs.astype(np.int64))).cpu().numpy()
        assert gh.astype(np.uint64).tolist() == oracle.window_hashes(s.text, 32, xs).tolist()
        # the hot-path kernel's own rolling hashes (single-bucket kernel, the
        # tuned geometry and full grid the bench runs) of every 4099th window
        stride = 4099
        d = bench_ctx.scan_dump(text, 32, stride, kernel=1).cpu().numpy().astype(np.uint64)
        xs = np.arange(0, s.text.size - 32 + 1, stride, dtype=np.uint64)
        assert d.size == xs.size > 10 ** 6
        assert np.array_equal(d, oracle.window_hashes(s.text, 32, xs))


@pytest.mark.parametrize("mode", MODES)
def test_config3_full_size(bench_ctx, rk, mode):
    """Config 3 at its full size (1 GiB Zipf text, 1,024 patterns of m=16),
    element by element against the threaded oracle."""
    s = rkgen.config3()
    got = run(bench_ctx, rk, s.text, s.patterns, mode)
    ref = oracle.search(s.text, s.patterns, threads=THREADS)
    assert int(ref[0][-1]) > 10 ** 6
    assert_same(got, ref, "config3 full " + mode)


@pytest.mark.parametrize("mode", MODES)
def test_config3_reduced_multi(ctx, rk, mode):
    s = rkgen.config3(n=(1 << 22) + 5, k=256, sampled=128)
    got = run(ctx, rk, s.text, s.patterns, mode)
    ref = oracle.search(s.text, s.patterns, threads=4)
    assert int(ref[0][-1]) > 1000
    assert_same(got, ref, "config3 " + mode)


@pytest.mark.parametrize("mode", MODES)
def test_random_small(ctx, rk, mode):
    g = rkgen.rng(50, 1 if mode == "screen" else 2)
    tables = [np.frombuffer(b"ab", np.uint8), rkgen.ACGT, rkgen.LOWER, rkgen.BYTE256]
    for trial in range(40):
        n = int(g.integers(0, 6000))
        table = tables[trial % 4]
        text = rkgen.iid_text(g, n, table)
        k = int(g.integers(0, 10))
        pats = []
        for _ in range(k):
            m = int(g.integers(1, 65))
            if n >= m and g.random() < 0.7:
                o = int(g.integers(0, n - m + 1))
                pats.append(text[o:o + m].tobytes())
            else:
                pats.append(rkgen.iid_text(g, m, table).tobytes())
        got = run(ctx, rk, text, pats, mode)
        assert_same(got, oracle.search(text, pats), "trial %d n=%d" % (trial, n))


@pytest.mark.parametrize("mode", MODES)
def test_many_patterns_per_length(ctx, rk, mode):
    """Hash-table buckets: dozens of distinct patterns per length, lengths
    1..3 (masked screen hashes) as well as longer ones, sampled and random,
    over small and large alphabets."""
    g = rkgen.rng(52, 1 if mode == "screen" else 2)
    for trial, table in enumerate([rkgen.ACGT, rkgen.LOWER, rkgen.BYTE256]):
        n = 200000
        text = rkgen.iid_text(g, n, table)
        pats = []
        for m in (1, 2, 3, 4, 5, 7, 8, 12, 16, 17, 31, 64):
            for j in range(40):
                if j % 2 == 0:
                    o = int(g.integers(0, n - m + 1))
                    pats.append(text[o:o + m].tobytes())
                else:
                    pats.append(rkgen.iid_text(g, m, table).tobytes())
        got = run(ctx, rk, text, pats, mode)
        assert_same(got, oracle.search(text, pats, threads=4), "trial %d" % trial)


@pytest.mark.parametrize("mode", MODES)
def test_large_pattern_set(ctx, rk, mode):
    """Thousands of patterns of mixed lengths in one plan (several table
    buckets and cuckoo tables, patterns read from device memory)."""
    g = rkgen.rng(53, 1 if mode == "screen" else 2)
    n = 1 << 20
    text = rkgen.iid_text(g, n, rkgen.LOWER)
    pats = []
    for j in range(6000):
        m = int(g.integers(4, 65))
        if j % 3 == 0:
            o = int(g.integers(0, n - m + 1))
            pats.append(text[o:o + m].tobytes())
        else:
            pats.append(rkgen.iid_text(g, m, rkgen.LOWER).tobytes())
    pats += pats[:50]  # duplicates: each copy gets the full list
    got = run(ctx, rk, text, pats, mode)
    assert_same(got, oracle.search(text, pats, threads=8), mode)


@pytest.mark.parametrize("mode", MODES)
def test_shared_keys_and_identical_runs(ctx, rk, mode):
    """Patterns of several lengths in one length class share the class's key
    (the hash of their last l bytes, l the class's shortest length): sets
    whose members end in the same bytes form runs of different patterns under
    one key, and copies of one pattern form runs of one pattern under several
    ids; both against the oracle, with hits dense enough that every tile has
    candidates."""
    g = rkgen.rng(57, 0 if mode == "screen" else 1)
    n = 1 << 20
    text = rkgen.iid_text(g, n, rkgen.ACGT)
    pats = []
    for o in g.integers(0, n - 64, size=40):
        o = int(o)
        for m in (4, 5, 7, 9, 12, 15, 16, 20, 31, 33, 48, 64):
            pats.append(text[o + 64 - m:o + 64].tobytes())  # all end at the same byte
    pats += pats[:30] * 3  # one pattern under four ids
    pats += [b"ACGT", b"ACGT", b"CGTA"]
    got = run(ctx, rk, text, pats, mode)
    assert_same(got, oracle.search(text, pats, threads=8), mode)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
def test_tile_seams_every_geometry(ctx, rk, mode, cfg):
    """Occurrences planted across tile and thread seams, first and last window."""
    lib = rk._lib.load()
    wg, c, tb = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    lib.rk_tile_cfg(cfg, ctypes.byref(wg), ctypes.byref(c), ctypes.byref(tb))
    W, C = tb.value, c.value
    g = rkgen.rng(51, cfg)
    n = 3 * W + 40
    text = rkgen.iid_text(g, n, rkgen.ACGT)
    pats = [rkgen.ACGT[g.integers(0, 4, size=m)].tobytes() for m in (1, 3, 4, 7, 16, 31, 32, 33, 63, 64)]
    for j, p in enumerate(pats):
        m = len(p)
        for base in (0, W, 2 * W, 3 * W, C, W + 5 * C, n - m):
            for d in (-m, -m + 1, -1, 0, 1):
                x = base + d
                if 0 <= x <= n - m:
                    text[x:x + m] = np.frombuffer(p, np.uint8)
    got = run(ctx, rk, text, pats, mode, {rk._lib.RK_OPT_TILE_CFG: cfg})
    assert_same(got, oracle.search(text, pats), "cfg %d" % cfg)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
@pytest.mark.parametrize("grid", [1, 7, 0])
def test_single_pattern_tile_pipeline(ctx, rk, mode, cfg, grid):
    """One pattern (the single-bucket kernel) in every geometry: with a small
    forced grid each workgroup walks many tiles through its LDS slots, so
    every slot is reused; occurrences sit across tile and thread seams and at
    both ends of a ragged text."""
    lib = rk._lib.load()
    wg, c, tb = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    lib.rk_tile_cfg(cfg, ctypes.byref(wg), ctypes.byref(c), ctypes.byref(tb))
    W, C = tb.value, c.value
    g = rkgen.rng(53, cfg * 3 + grid % 5)
    n = 37 * W + 91
    text = rkgen.iid_text(g, n, rkgen.ACGT)
    m = (32, 5, 17, 64)[cfg]
    p = rkgen.ACGT[g.integers(0, 4, size=m)].tobytes()
    for k in range(38):
        for d in (-m, -m + 1, -1, 0, 1, C - 1, 3 * C + 2):
            x = k * W + d
            if 0 <= x <= n - m:
                text[x:x + m] = np.frombuffer(p, np.uint8)
    text[n - m:] = np.frombuffer(p, np.uint8)
    opts = {rk._lib.RK_OPT_TILE_CFG: cfg}
    if grid:
        opts[rk._lib.RK_OPT_GRID] = grid
    got = run(ctx, rk, text, [p], mode, opts)
    ref = oracle.search(text, [p])
    assert int(ref[0][-1]) > 30  # overlapping plants of the long patterns overwrite each other
    assert_same(got, ref, "cfg %d grid %d" % (cfg, grid))


@pytest.mark.parametrize("mode", MODES)
def test_edge_cases(ctx, rk, mode):
    cases = [
        (b"abcab", [b"ab"]),
        (b"abc", [b"abc", b"abcd"]),
        (b"aaaa", [b"aa", b"a"]),
        (b"\x00\xff\x00\xff\x00", [b"\x00\xff", b"\xff\x00\xff"]),
        (b"xyxyx", [b"yx", b"yx"]),
        (b"abc", []),
        (b"", [b"a"]),
        (b"a" * 5000, [b"a" * 64, b"a" * 33, b"a"]),
        (b"\x00" * 3000, [b"\x00" * 9, b"\x00\x01"]),
    ]
    for text, pats in cases:
        got = run(ctx, rk, np.frombuffer(text, np.uint8), pats, mode)
        assert_same(got, oracle.search(text, pats), repr((text[:10], pats[:2])))


@pytest.mark.parametrize("mode", MODES)
def test_constructed_collisions_are_rejected(ctx, rk, mode):
    """Windows with the pattern's d=256 hash but other bytes are not reported,
    and the scan's own rolling hashes of both windows are equal."""
    g = rkgen.rng(52, 0)
    text = rkgen.iid_text(g, 100000, rkgen.LOWER)
    pats = []
    for m in (9, 16, 40, 64):
        w = bytearray(rkgen.LOWER[g.integers(8, 18, size=m)].tobytes())
        w2 = bytearray(w)
        w2[0] += 1
        w2[8] -= 8
        assert oracle.hash(bytes(w)) == oracle.hash(bytes(w2))
        for x in range(1000 * m, 1000 * m + 10 * m, m):
            text[x:x + m] = np.frombuffer(bytes(w2), np.uint8)
        text[200 * m:200 * m + m] = np.frombuffer(bytes(w), np.uint8)
        pats.append(bytes(w))
    got = run(ctx, rk, text, pats, mode)
    ref = oracle.search(text, pats)
    assert_same(got, ref, "collisions")
    assert int(ref[0][-1]) == len(pats)
    # the dumped rolling hashes of w and w2 windows agree
    t = dev(text)
    for w in pats:
        m = len(w)
        for kernel in (0, 1):
            d = ctx.scan_dump(t, m, m, kernel=kernel).cpu().numpy().astype(np.uint64)
            assert d[200] == d[1000] == np.uint64(oracle.hash(w))


@pytest.mark.parametrize("kernel", [0, 1])
def test_scan_dump_matches_oracle(ctx, rk, kernel):
    """Every length 1..64 (so every out-term specialisation of the rolling
    step: r = 8m mod 61 in the low word, in the high word, or anywhere): the
    hashes a scan kernel's own rolling loop holds for sampled windows equal the
    oracle's direct evaluation.  kernel 0 = general scan, 1 = single-bucket."""
    g = rkgen.rng(53, kernel)
    n = 300000 + 13
    text = np.frombuffer(g.bytes(n), np.uint8).copy()
    t = dev(text)
    stride = 997
    for m in range(1, 65):
        d = ctx.scan_dump(t, m, stride, kernel=kernel).cpu().numpy().astype(np.uint64)
        xs = np.arange(0, n - m + 1, stride, dtype=np.uint64)
        assert d.tolist() == oracle.window_hashes(text, m, xs).tolist(), "m=%d" % m


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
def test_scan_dump_every_geometry(ctx, rk, kernel, cfg):
    """The dump in every tile geometry with a forced small grid (each
    workgroup walks many tiles, reusing both LDS slots), stride 1 around tile
    seams and a ragged end: one kernel's rolling state equals direct Horner."""
    lib = rk._lib.load()
    wg, c, tb = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    lib.rk_tile_cfg(cfg, ctypes.byref(wg), ctypes.byref(c), ctypes.byref(tb))
    W = tb.value
    g = rkgen.rng(55, cfg)
    n = 9 * W + 45
    text = np.frombuffer(g.bytes(n), np.uint8).copy()
    t = dev(text)
    ctx.set_option(rk._lib.RK_OPT_TILE_CFG, cfg)
    ctx.set_option(rk._lib.RK_OPT_GRID, 3)
    try:
        for m in (4, 7, 32, 64):
            d = ctx.scan_dump(t, m, 1, kernel=kernel).cpu().numpy().astype(np.uint64)
            xs = np.arange(0, n - m + 1, dtype=np.uint64)
            assert d.tolist() == oracle.window_hashes(text, m, xs).tolist(), "m=%d" % m
    finally:
        ctx.set_option(rk._lib.RK_OPT_TILE_CFG, -1)
        ctx.set_option(rk._lib.RK_OPT_GRID, 0)


def test_window_hashes_match_oracle(ctx, rk):
    g = rkgen.rng(54, 0)
    n = 100000
    text = np.frombuffer(g.bytes(n), np.uint8).copy()
    t = dev(text)
    for m in (1, 8, 9, 32, 64, 100, 800):
        xs = np.unique(g.integers(0, n - m + 1, size=500)).astype(np.int64)
        got = ctx.window_hashes(t, m, torch.from_numpy(xs)).cpu().numpy().astype(np.uint64)
        assert got.tolist() == oracle.window_hashes(text, m, xs.astype(np.uint64)).tolist()
    bad = ctx.window_hashes(t, 10, torch.tensor([n - 9, n], dtype=torch.int64)).cpu().numpy()
    assert (bad.astype(np.uint64) == np.uint64(2**64 - 1)).all()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("k", [1, 3])
def test_sparse_compaction_clustered_hits(ctx, rk, mode, k):
    """Fewer hits than tiles, so the collect compacts a tile per lane: most
    tiles hold 0-2 hits (a lane copies them), a cluster of 20 plants puts
    more than eight in one tile (the wave copies it), and a dense cluster
    overflows its tile's staging slab (rescanned, not compacted)."""
    g = rkgen.rng(56, k)
    n = (64 if k == 1 else 128) << 20
    text = rkgen.iid_text(g, n, np.frombuffer(b"ACGT", np.uint8))
    p0 = np.frombuffer(b"ACGTTGCAAC", np.uint8)
    # more plants in one tile than its slab holds: W/64 records for a single
    # pattern (up to 528 at W = 33,792), W/16 for a set (up to 2,112)
    span, step = (16384, 20) if k == 1 else (24576, 10)
    for o in range(1 << 20, (1 << 20) + span - 10, step):
        text[o:o + 10] = p0
    for o in range(9 << 20, (9 << 20) + 20 * 64, 64):
        text[o:o + 10] = p0
    pats = [p0.tobytes()] + [bytes(g.choice(np.frombuffer(b"ACGT", np.uint8), 10)) for _ in range(k - 1)]
    ref = oracle.search(text, pats, threads=4)
    assert int(ref[0][-1]) < n // (256 * 132)  # fewer hits than tiles, whatever the geometry
    assert_same(run(ctx, rk, text, pats, mode), ref, "clustered k=%d %s" % (k, mode))


@pytest.mark.parametrize("k", [1, 2])
def test_tile_offsets_beyond_256_sum_blocks(ctx, rk, k):
    """A 10 GiB text in the 9,216-byte tile geometry has 1,165,085 tiles, more
    than 256 blocks of 4,096: the collect then scans the count pass's block
    sums in one workgroup before the per-block tile offsets.  The text is one
    byte repeated with plants 64 bytes apart or more, so the positions are
    known without the oracle."""
    n = 10 << 30
    assert (n + 9215) // 9216 > 256 * 4096
    g = rkgen.rng(57, k)
    pats = [b"xyzzy", b"qqq"][:k]
    text = torch.full((n,), ord("a"), dtype=torch.uint8, device="cuda:0")
    try:
        want = []
        for j, p in enumerate(pats):
            # spread over the whole text, plus the first and the last windows
            pos = np.unique(g.integers(0, n // 64 - 1, size=3000)) * 64 + 16 * j
            pos = np.concatenate([[j * 8], pos, [n - len(p) - 32 * j]]).astype(np.int64)
            pos = np.unique(pos)
            idx = torch.from_numpy(pos).to("cuda:0")
            for i, c in enumerate(p):
                text[idx + i] = c
            want.append(pos)
        torch.cuda.synchronize()
        ctx.set_option(rk._lib.RK_OPT_TILE_CFG, 3)
        try:
            plan = rk.Plan(ctx, pats, "screen")
            off, got = plan.search(text)
            torch.cuda.synchronize()
            plan.close()
        finally:
            ctx.set_option(rk._lib.RK_OPT_TILE_CFG, -1)
        off = off.cpu().numpy()
        got = got.cpu().numpy()
        for j in range(k):
            assert got[off[j]:off[j + 1]].tolist() == want[j].tolist(), j
    finally:
        del text
        torch.cuda.empty_cache()


def test_stream_read_folds_every_word_once(ctx, rk):
    """The roofline's read kernel: the XOR of its per-workgroup folds is the
    XOR of every 4-byte word of the buffer (a chunk read twice or skipped
    would change it), for grids that leave waves idle, bodies that are not a
    whole number of batches and a tail that is not a whole 1 KiB chunk."""
    import ctypes
    g = rkgen.rng(55, 0)
    for n in (16, 1008, 1024, (1 << 20) + 528, 8 * 1024 * 37 + 16 * 5):
        data = np.frombuffer(g.bytes(n), np.uint8).copy()
        want = int(np.bitwise_xor.reduce(data.view(np.uint32)))
        t = dev(data)
        for grid in (1, 7, 64, 300):
            out = torch.zeros(grid, dtype=torch.int32, device="cuda:0")
            st = ctx.lib.rk_stream_read(ctx.h, ctypes.c_void_p(t.data_ptr()), n, ctypes.c_void_p(out.data_ptr()),
                                        grid, None)
            assert st == 0
            torch.cuda.synchronize()
            got = int(np.bitwise_xor.reduce(out.cpu().numpy().view(np.uint32)))
            assert got == want, (n, grid)


@pytest.mark.parametrize("mode", MODES)
def test_slab_overflow_rescan(ctx, rk, mode):
    """A one-slot staging slab forces every tile with hits through the rescan."""
    s = rkgen.config3(n=1 << 20, k=64, sampled=48)
    got = run(ctx, rk, s.text, s.patterns, mode, {rk._lib.RK_OPT_SLAB_CAP: 1})
    assert_same(got, oracle.search(s.text, s.patterns, threads=4), "slab=1")


@pytest.mark.parametrize("mode", MODES)
def test_queue_and_grid_options(ctx, rk, mode):
    s = rkgen.config2(n=(1 << 21) + 3, plants=100)
    ref = oracle.search(s.text, s.patterns)
    for opts in ({rk._lib.RK_OPT_QUEUE: 1}, {rk._lib.RK_OPT_GRID: 7}, {rk._lib.RK_OPT_QUEUE: 1,
                                                                        rk._lib.RK_OPT_GRID: 3}):
        assert_same(run(ctx, rk, s.text, s.patterns, mode, opts), ref, str(opts))


LONG = (65, 100, 200, 800, 1024)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
def test_long_patterns_seams(ctx, rk, mode, cfg):
    """Patterns longer than the rolled window (65..1024 bytes): occurrences
    planted across tile and thread seams, at both ends of a ragged text, and
    overlapping; one plan with all lengths plus short ones (multi-bucket
    kernel) and each long pattern alone (single-bucket kernel), with a small
    grid so every workgroup walks many tiles."""
    lib = rk._lib.load()
    wg, c, tb = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    lib.rk_tile_cfg(cfg, ctypes.byref(wg), ctypes.byref(c), ctypes.byref(tb))
    W, C = tb.value, c.value
    g = rkgen.rng(57, cfg)
    n = 5 * W + 1500
    text = rkgen.iid_text(g, n, rkgen.ACGT)
    pats = [rkgen.ACGT[g.integers(0, 4, size=m)].tobytes() for m in LONG]
    for j, p in enumerate(pats):
        m = len(p)
        for base in (0, W, 2 * W + C, 4 * W, n - m):
            for d in (-m, -m + 1, -1, 0, 1, j):
                x = base + d
                if 0 <= x <= n - m:
                    text[x:x + m] = np.frombuffer(p, np.uint8)
    # short patterns and a long one that shares the last 64 bytes of another
    extra = [text[10:18].tobytes(), text[W - 20:W + 12].tobytes(), b"G" * 3 + pats[3][3:]]
    opts = {rk._lib.RK_OPT_TILE_CFG: cfg, rk._lib.RK_OPT_GRID: 5}
    allp = pats + extra
    got = run(ctx, rk, text, allp, mode, opts)
    ref = oracle.search(text, allp)
    assert int(ref[0][-1]) > 10  # plants of the long patterns overwrite each other
    assert_same(got, ref, "long cfg %d" % cfg)
    for p in pats:
        assert_same(run(ctx, rk, text, [p], mode, opts), oracle.search(text, [p]), "single m=%d" % len(p))


@pytest.mark.parametrize("mode", MODES)
def test_long_patterns_random(ctx, rk, mode):
    """Random texts over four alphabets with mixed short and long patterns
    (sampled and random), duplicates, runs of one byte (every window of a
    long run matches), against the oracle."""
    g = rkgen.rng(58, 1 if mode == "screen" else 2)
    tables = [np.frombuffer(b"ab", np.uint8), rkgen.ACGT, rkgen.LOWER, rkgen.BYTE256]
    for trial in range(24):
        n = int(g.integers(0, 30000))
        table = tables[trial % 4]
        text = rkgen.iid_text(g, n, table)
        if trial % 6 == 5 and n > 3000:
            text[1000:2500] = table[0]
        pats = []
        for _ in range(int(g.integers(1, 12))):
            m = int(g.choice([3, 16, 64, 65, 66, 127, 128, 300, 700, 1024]))
            if n >= m and g.random() < 0.7:
                o = int(g.integers(0, n - m + 1))
                pats.append(text[o:o + m].tobytes())
            else:
                pats.append(rkgen.iid_text(g, m, table).tobytes())
        if trial % 6 == 5:
            pats += [bytes([table[0]]) * 200, bytes([table[0]]) * 1024]
        pats += pats[:1]
        got = run(ctx, rk, text, pats, mode)
        assert_same(got, oracle.search(text, pats), "trial %d n=%d" % (trial, n))


@pytest.mark.parametrize("mode", MODES)
def test_count_per_pattern(ctx, rk, mode):
    """rk_count's per-pattern counts equal the oracle's list lengths: a
    multi-pattern plan (table buckets), one pattern (the single-bucket
    kernel), a few patterns sharing register targets, duplicates, and a
    one-slot slab (every tile with hits overflows: counts still complete)."""
    s = rkgen.config3(n=(1 << 21) + 9, k=96, sampled=64)
    g = rkgen.rng(56, 0)
    cases = [(s.text, s.patterns, {}), (s.text, s.patterns[:1], {}), (s.text, s.patterns[:3] + s.patterns[:2], {}),
             (s.text, s.patterns, {rk._lib.RK_OPT_SLAB_CAP: 1})]
    text4 = rkgen.iid_text(g, 70000, rkgen.ACGT)
    cases.append((text4, [text4[100:104].tobytes(), b"A", b"ACGTACGTAC"], {}))
    for i, (text_np, pats, opts) in enumerate(cases):
        ro, _ = oracle.search(text_np, pats, threads=4)
        for k, v in opts.items():
            ctx.set_option(k, v)
        try:
            plan = rk.Plan(ctx, pats, mode)
            t = dev(text_np)
            counts = torch.full((len(pats),), -5, dtype=torch.int64, device="cuda:0")
            total = plan.count(t, counts=counts)
            plan.close()
        finally:
            for k in opts:
                ctx.set_option(k, 0)
        assert total == int(ro[-1]), i
        assert counts.cpu().numpy().astype(np.uint64).tolist() == np.diff(ro).tolist(), i


def test_errors(ctx, rk):
    RkError = rk._lib.RkError
    with pytest.raises(RkError) as e:
        rk.Plan(ctx, [b""])
    assert e.value.status == rk._lib.RK_EINVAL
    with pytest.raises(RkError) as e:
        rk.Plan(ctx, [b"a" * 1025])
    assert e.value.status == rk._lib.RK_EUNSUPPORTED
    text = dev(np.zeros(4096, np.uint8))
    plan = rk.Plan(ctx, [b"\x00\x00"])
    with pytest.raises(RkError) as e:
        plan.count(text[1:])
    assert e.value.status == rk._lib.RK_EINVAL
    total = plan.count(text)
    assert total == 4095
    with pytest.raises(RkError) as e:
        plan.collect(text, total, out=(torch.empty(2, dtype=torch.int64, device="cuda:0"),
                                       torch.empty(10, dtype=torch.int64, device="cuda:0")))
    assert e.value.status == rk._lib.RK_ENOSPACE
    small = torch.empty(16, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(RkError) as e:
        plan.count(text, scratch=small)
    assert e.value.status == rk._lib.RK_ENOSPACE
    plan.close()


@pytest.mark.parametrize("mode", MODES)
def test_batch_matches_solo_and_oracle(ctx, rk, mode):
    insts = rkgen.config4(count=24, lmax=1 << 18)
    texts = [dev(s.text) for s in insts]
    bp = rk.BatchPlan(ctx, texts, [s.patterns for s in insts], mode)
    off, pos = bp.search()
    torch.cuda.synchronize()
    per = bp.split(off, pos)
    for i, s in enumerate(insts):
        ro, rp = oracle.search(s.text, s.patterns)
        ref = oracle.split(ro, rp)
        for j in range(len(s.patterns)):
            assert per[i][j].astype(np.uint64).tolist() == ref[j].tolist(), (i, j)
        solo = run(ctx, rk, s.text, s.patterns, mode)
        assert_same(solo, (ro, rp), "solo %d" % i)
    bp.close()


@pytest.fixture(scope="module")
def config4_full():
    """Config 4 at its full size (4,096 instances, log-uniform 4 KiB..16 MiB,
    alphabets 4/26/256, 1..32 patterns of 4..64 bytes) with the oracle's
    per-pattern lists of every instance (instances in parallel)."""
    from concurrent.futures import ThreadPoolExecutor
    insts = rkgen.config4()
    with ThreadPoolExecutor(THREADS) as ex:
        refs = list(ex.map(lambda s: oracle.split(*oracle.search(s.text, s.patterns)), insts))
    return insts, refs


@pytest.mark.parametrize("mode", MODES)
def test_config4_full_size(bench_ctx, rk, config4_full, mode):
    """Every instance of the full config-4 batch: the batched result (one
    persistent launch over the bucketed work queue, the bench's tuning
    table) equals the oracle's, and so does each instance searched alone."""
    insts, refs = config4_full
    offs, o = [], 0
    for s in insts:
        offs.append(o)
        o += (len(s.text) + 255) // 256 * 256
    buf = torch.empty(o, dtype=torch.uint8, device="cuda:0")
    for s, off in zip(insts, offs):
        buf[off:off + len(s.text)].copy_(torch.from_numpy(s.text))
    texts = [buf[off:off + len(s.text)] for s, off in zip(insts, offs)]
    bp = rk.BatchPlan(bench_ctx, texts, [s.patterns for s in insts], mode)
    off_b, pos_b = bp.search()
    torch.cuda.synchronize()
    per = bp.split(off_b, pos_b)
    bp.close()
    bad = [(i, j) for i, s in enumerate(insts) for j in range(len(s.patterns))
           if per[i][j].astype(np.uint64).tolist() != refs[i][j].tolist()]
    assert not bad, "batched != oracle at %s" % bad[:5]
    for i, s in enumerate(insts):
        plan = rk.Plan(bench_ctx, s.patterns, mode)
        so, sp = plan.search(texts[i])
        lists = oracle.split(so.cpu().numpy().astype(np.uint64), sp.cpu().numpy().astype(np.uint64))
        plan.close()
        for j in range(len(s.patterns)):
            assert lists[j].tolist() == refs[i][j].tolist(), ("solo", i, j)
    del buf
