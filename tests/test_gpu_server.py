"""Serving: every request's result is the same alone (a solo search through
the C ABI, and the CPU oracle) and in the mix (merged steps, several steps in
flight, graph replays, admission waits on a small arena).  Exact equality."""
import time

import numpy as np
import pytest

import oracle
import rkgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def corpora():
    cs = [rkgen.config5_corpus(i, n=(1 << 20) + 64 * i) for i in range(4)]
    torch.cuda.synchronize()
    return cs


def make_requests(corpora, count, seed, kmax=24):
    host = [c.cpu().numpy() for c in corpora]

    def sample(ci, g, m):
        o = int(g.integers(0, len(host[ci]) - m + 1))
        return host[ci][o:o + m].tobytes()

    reqs = rkgen.config5_requests(rate=1000.0, duration=count / 1000.0, corpora=len(corpora), kmax=kmax,
                                  sample_text=sample, seed_sub=seed)
    return reqs, host


def solo(ctx, rk, text, pats, mode):
    plan = rk.Plan(ctx, pats, mode)
    off, pos = plan.search(text)
    torch.cuda.synchronize()
    plan.close()
    return off.cpu().numpy().astype(np.uint64), pos.cpu().numpy().astype(np.uint64)


@pytest.mark.parametrize("mode,graphs,inflight,arena", [
    ("screen", True, 2, 1 << 28),
    ("screen", False, 3, 1 << 28),
    ("exact", True, 2, 1 << 28),
    ("screen", True, 3, 1 << 26),  # smaller arena: counted steps may wait for memory
])
def test_mix_equals_solo_and_oracle(ctx, rk, corpora, mode, graphs, inflight, arena):
    reqs, host = make_requests(corpora, 48, seed=7)
    assert len(reqs) > 20
    srv = rk.Server(ctx, arena_bytes=arena, max_inflight=inflight, max_step_requests=5, mode=mode,
                    use_graphs=graphs)
    ids = [srv.add_corpus(c) for c in corpora]
    assert ids == list(range(len(corpora)))
    rids = []
    for r in reqs:
        rids.append(srv.submit(r.corpus, r.patterns))
        time.sleep(0.0005)
    srv.drain()
    st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["steps"] >= len(reqs) // 5
    for i, (r, rid) in enumerate(zip(reqs, rids)):
        res = srv.wait(rid)
        assert res["status"] == 0
        so, sp = solo(ctx, rk, corpora[r.corpus], r.patterns, mode)
        assert res["offsets"].tolist() == so.tolist(), i
        assert res["positions"].tolist() == sp.tolist(), i
        if i % 6 == 0:
            ro, rp = oracle.search(host[r.corpus], r.patterns, threads=4)
            assert res["offsets"].tolist() == ro.tolist() and res["positions"].tolist() == rp.tolist(), i
        srv.release(rid)
    srv.close()


def test_duplicate_patterns_across_requests(ctx, rk, corpora):
    """Two requests sharing patterns in one step each get their own full lists."""
    text = corpora[0]
    h = text.cpu().numpy()
    a = [h[100:108].tobytes(), h[5000:5016].tobytes(), b"zzzzqqqq"]
    b = [h[5000:5016].tobytes(), h[100:108].tobytes(), h[100:108].tobytes()]
    srv = rk.Server(ctx, max_inflight=1, max_step_requests=8)
    srv.add_corpus(text)
    pairs = [(srv.submit(0, a), srv.submit(0, b)) for _ in range(8)]
    srv.drain()
    st = srv.stats()
    # identical patterns of requests that share a step are searched once
    assert st["merged_patterns"] <= st["request_patterns"]
    ra, rb = pairs[-1]
    xa, xb = srv.wait(ra), srv.wait(rb)
    oa, pa = oracle.search(h, a)
    ob, pb = oracle.search(h, b)
    assert xa["offsets"].tolist() == oa.tolist() and xa["positions"].tolist() == pa.tolist()
    assert xb["offsets"].tolist() == ob.tolist() and xb["positions"].tolist() == pb.tolist()
    srv.close()


def test_cancel_and_errors(ctx, rk, corpora):
    srv = rk.Server(ctx, max_inflight=1, max_step_requests=1)
    srv.add_corpus(corpora[1])
    rids = [srv.submit(0, [b"abcd", b"e f"]) for _ in range(30)]
    canceled = sum(1 for r in rids[10:] if srv.cancel(r) == 0)
    srv.drain()
    st = srv.stats()
    assert st["completed"] + st["canceled"] == 30 and st["canceled"] == canceled
    with pytest.raises(rk._lib.RkError):
        srv.submit(5, [b"x"])  # unknown corpus
    with pytest.raises(rk._lib.RkError):
        srv.submit(0, [b""])
    empty = srv.wait(srv.submit(0, []))
    assert empty["status"] == 0 and empty["offsets"].tolist() == [0]
    srv.close()


def test_oversized_steps_are_split(ctx, rk, corpora):
    """A step whose merged output does not fit the arena goes back to the
    queue and is split; every request still gets its exact result.  The arena
    holds one request's output and sort work (about 19 bytes per hit) but not
    two, so any step of two or more requests must be split."""
    text = corpora[2]
    h = text.cpu().numpy()
    # one- and two-byte patterns: each request has many hits, so the fixed
    # part of a step's need (offsets, radix histograms) is small beside them
    pats = [h[o:o + m].tobytes() for o, m in ((10, 1), (2000, 1), (40000, 2), (123456, 1))]
    reqs = [pats[i % 4:] + pats[:i % 4] for i in range(12)]
    ref = [oracle.search(h, r) for r in reqs]
    hits = int(ref[0][0][-1])
    assert hits > 20000
    srv = rk.Server(ctx, arena_bytes=30 * hits, max_inflight=1, max_step_requests=64)
    srv.add_corpus(text)
    rids = [srv.submit(0, r) for r in reqs]
    # results are released as they are checked: unreleased results hold arena
    # space that later steps wait for
    for i, rid in enumerate(rids):
        res = srv.wait(rid)
        assert res["status"] == 0, i
        assert res["offsets"].tolist() == ref[i][0].tolist(), i
        assert res["positions"].tolist() == ref[i][1].tolist(), i
        srv.release(rid)
    srv.drain()
    st = srv.stats()
    assert st["completed"] == 12 and st["failed"] == 0
    # no split means every step held a single request
    assert st["step_splits"] >= 1 or st["steps"] == 12, st
    srv.close()


def test_completion_queue(ctx, rk, corpora):
    """next_done reports every finished request once (done or canceled), in
    completion order; results consumed and released that way equal solo
    searches."""
    reqs, host = make_requests(corpora, 40, seed=11)
    srv = rk.Server(ctx, arena_bytes=1 << 27, max_inflight=2, max_step_requests=6)
    for c in corpora:
        srv.add_corpus(c)
    rids = [srv.submit(r.corpus, r.patterns) for r in reqs]
    canceled = {r for r in rids[-6:] if srv.cancel(r) == 0}
    seen, done_times, got = [], [], {}
    while len(seen) < len(rids):
        rid = srv.next_done(timeout=60.0)
        assert rid is not None, "no completion within 60 s"
        seen.append(rid)
        res = srv.wait(rid, timeout=0.0)
        if rid in canceled:
            assert res["status"] == rk._lib.RK_ECANCELED
        else:
            assert res["status"] == 0
            done_times.append(res["t_done"])
            got[rid] = (res["offsets"].tolist(), res["positions"].tolist())
        srv.release(rid)
    assert sorted(seen) == sorted(rids)
    assert done_times == sorted(done_times)
    assert srv.next_done(timeout=0.05) is None
    srv.close()
    for i, rid in enumerate(rids):
        if rid in canceled:
            continue
        r = reqs[i]
        so, sp = solo(ctx, rk, corpora[r.corpus], r.patterns, "screen")
        assert got[rid] == (so.tolist(), sp.tolist()), i


def test_dense_steps_size_their_slabs(ctx, rk, corpora):
    """Merged steps of dense short patterns: once the server has a hit-rate
    estimate it sizes each step's staging slabs from it (more records per tile
    than the default), and every result still equals the oracle's, in both
    modes and with several steps in flight."""
    text = corpora[3]
    h = text.cpu().numpy()
    offs = (7, 333, 4096, 70000, 250000, 600000)
    reqs = [[h[o:o + m].tobytes() for o, m in zip(offs[i % 3:i % 3 + 4], (1, 2, 1, 3))] for i in range(18)]
    ref = [oracle.search(h, r) for r in reqs]
    assert min(int(r[0][-1]) for r in ref) > 10000
    for mode in ("screen", "exact"):
        srv = rk.Server(ctx, arena_bytes=1 << 30, max_inflight=3, max_step_requests=3, mode=mode)
        srv.add_corpus(text)
        rids = [srv.submit(0, r) for r in reqs]
        for i, rid in enumerate(rids):
            res = srv.wait(rid)
            assert res["status"] == 0, (mode, i)
            assert res["offsets"].tolist() == ref[i][0].tolist(), (mode, i)
            assert res["positions"].tolist() == ref[i][1].tolist(), (mode, i)
            srv.release(rid)
        st = srv.stats()
        assert st["completed"] == len(reqs) and st["failed"] == 0
        assert st["steps"] >= len(reqs) // 3
        srv.close()


def test_admission_wait_is_bounded(ctx, rk, corpora):
    """A client that holds every result unreleased fills the arena: a later
    step that finds no room while nothing else is in flight ends RK_ENOSPACE
    after the admission timeout instead of waiting forever; the requests
    admitted before it are exact, and releasing results lets new steps run."""
    text = corpora[2]
    h = text.cpu().numpy()
    pats = [h[o:o + m].tobytes() for o, m in ((10, 1), (2000, 1), (40000, 2))]
    ref = oracle.search(h, pats)
    hits = int(ref[0][-1])
    # a step needs about 19 bytes per hit of the arena (8 for the positions,
    # 8 for the records being sorted, the digit histograms); a finished,
    # unreleased result keeps its 8: 32 bytes per hit admit two steps and
    # leave the third without room
    srv = rk.Server(ctx, arena_bytes=32 * hits, max_inflight=1, max_step_requests=1, admission_timeout_s=0.2)
    srv.add_corpus(text)
    t0 = time.perf_counter()
    rids = [srv.submit(0, pats) for _ in range(4)]
    res = [srv.wait(r, timeout=30.0, fetch=False) for r in rids]
    assert time.perf_counter() - t0 < 20.0
    status = [r["status"] for r in res]
    assert status[0] == 0 and rk._lib.RK_ENOSPACE in status, status
    assert set(status) <= {0, rk._lib.RK_ENOSPACE}, status
    first = srv.wait(rids[0])
    assert first["offsets"].tolist() == ref[0].tolist() and first["positions"].tolist() == ref[1].tolist()
    for r in rids:
        srv.release(r)
    again = srv.wait(srv.submit(0, pats), timeout=30.0)
    assert again["status"] == 0 and again["positions"].tolist() == ref[1].tolist()
    srv.close()


def test_request_timeout(ctx, rk, corpora):
    """Requests that wait longer than the request timeout for a step end
    RK_ETIMEDOUT; the others are exact."""
    text = corpora[0]
    h = text.cpu().numpy()
    srv = rk.Server(ctx, max_inflight=1, max_step_requests=1, request_timeout_s=0.002)
    srv.add_corpus(text)
    reqs = [[h[o:o + 8].tobytes(), h[o + 50:o + 66].tobytes()] for o in range(0, 30000, 1000)]
    rids = [srv.submit(0, r) for r in reqs]
    srv.drain()
    timed_out = 0
    for r, rid in zip(reqs, rids):
        res = srv.wait(rid, timeout=0.0)
        if res["status"] == rk._lib.RK_ETIMEDOUT:
            timed_out += 1
            continue
        assert res["status"] == 0
        ro, rp = oracle.search(h, r)
        assert res["offsets"].tolist() == ro.tolist() and res["positions"].tolist() == rp.tolist()
        srv.release(rid)
    assert timed_out >= 1
    assert srv.stats()["failed"] >= timed_out
    srv.close()


class _DevView:
    """A device array of the server arena seen by torch (read only here)."""

    def __init__(self, ptr, n):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": "<u8", "data": (ptr, False), "version": 2}


def test_serving_full_size_corpora(ctx, rk):
    """Config 5 at its real sizes: 64 resident corpora of 1 GiB, Poisson
    request streams at 500, 2,000 and 8,000 req/s (a short window each), up
    to 256 patterns of 4..64 bytes per request.  Every result equals a solo
    search of the same request (compared on the device), and a seeded 1% of
    the requests equal the CPU oracle over the first 32 MiB of their corpus
    (the windows there; a whole-corpus oracle pass per distinct length would
    take minutes per request)."""
    import threading
    n = 1 << 30
    corpora = [rkgen.config5_corpus(i, n) for i in range(64)]
    torch.cuda.synchronize()
    srv = rk.Server(ctx, arena_bytes=48 << 30, max_inflight=2, mode="screen")
    for c in corpora:
        srv.add_corpus(c)
    pick = rkgen.rng(5, 777)
    checked = oracle_checked = 0
    # the checks run on a stream of their own: the server captures graphs on
    # its streams meanwhile, and work on the legacy stream must not wait on them
    side = torch.cuda.Stream()
    for rate, window in ((500.0, 0.4), (2000.0, 0.1), (8000.0, 0.03)):
        specs = rkgen.config5_request_specs(rate, window, n, corpora=64, seed_sub=int(rate) + 1)
        reqs = []
        for t, c, pats in specs:
            ps = [corpora[c][p[0]:p[0] + p[1]].cpu().numpy().tobytes() if isinstance(p, tuple) else p
                  for p in pats]
            reqs.append((t, c, ps))
        index = {}

        def submit():
            t0 = time.perf_counter()
            for i, (t, c, ps) in enumerate(reqs):
                d = t0 + t - time.perf_counter()
                if d > 0:
                    time.sleep(d)
                index[srv.submit(c, ps)] = i

        th = threading.Thread(target=submit)
        th.start()
        sample = set(pick.choice(len(reqs), size=max(1, len(reqs) // 100), replace=False).tolist())
        for _ in range(len(reqs)):
            rid = srv.next_done(timeout=120.0)
            assert rid is not None
            while rid not in index:
                time.sleep(0.0005)
            i = index[rid]
            t, c, ps = reqs[i]
            res = srv.wait(rid, timeout=0.0, fetch=False)
            assert res["status"] == 0, (rate, i)
            tot = int(res["offsets"][-1])
            with torch.cuda.stream(side):
                plan = rk.Plan(ctx, ps, "screen")
                so, sp = plan.search(corpora[c], stream=side)
                side.synchronize()
                plan.close()
                assert res["offsets"].tolist() == so.cpu().numpy().astype(np.uint64).tolist(), (rate, i)
                if tot:
                    got = torch.as_tensor(_DevView(res["positions_dev"], tot), device="cuda:0")
                    assert torch.equal(got.view(torch.int64), sp[:tot]), (rate, i)
                if i in sample:
                    # the oracle on the corpus's first 32 MiB (a request has up
                    # to 61 distinct lengths, one oracle pass each): the
                    # server's windows that lie in that prefix equal it
                    pre = 32 << 20
                    ro, rp = oracle.search(corpora[c][:pre].cpu().numpy(), ps, threads=16)
                    gp = sp.cpu().numpy().astype(np.uint64)
                    go = so.cpu().numpy().astype(np.int64)
                    for j, pat in enumerate(ps):
                        mine = gp[go[j]:go[j + 1]]
                        mine = mine[mine + len(pat) <= pre]
                        assert mine.tolist() == rp[ro[j]:ro[j + 1]].tolist(), (rate, i, j)
                    oracle_checked += 1
            srv.release(rid)
            checked += 1
        th.join()
    st = srv.stats()
    assert st["failed"] == 0 and st["completed"] == checked
    assert oracle_checked >= 3
    srv.close()
    del corpora
