"""The paper's GPU procedure (paper mode, rk_paper_search) against the
oracle: every window's 32-bit shift-add hash (d = 2, q = 2^32) equals the
oracle's direct evaluation, and the result array marks exactly the oracle's
match positions, for every threads-per-block value of the paper's tables."""
import numpy as np
import pytest

import oracle
import rkgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TPB = (32, 64, 128, 256, 512, 1024)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1810_01051_amd as rk
    c = rk.Context(0)
    yield c
    c.close()


def expect_flags(text, pat):
    nwin = max(len(text) - len(pat) + 1, 0)
    f = np.zeros(nwin, np.uint8)
    ro, rp = oracle.search(text, [pat])
    f[rp.astype(np.int64)] = 1
    return f


@pytest.mark.parametrize("tpb", TPB)
def test_paper_mode_hashes_and_matches(ctx, tpb):
    g = rkgen.rng(70, tpb)
    tables = [rkgen.ACGT, rkgen.LOWER, rkgen.BYTE256]
    for trial in range(12):
        n = int(g.integers(1, 50000))
        table = tables[trial % 3]
        text = rkgen.iid_text(g, n, table)
        m = int(g.choice([1, 2, 7, 16, 25, 31, 32, 33, 50, 100, 200, 800]))
        if n >= m and trial % 2 == 0:
            o = int(g.integers(0, n - m + 1))
            pat = text[o:o + m].tobytes()
            for x in g.integers(0, n - m + 1, size=5):
                text[x:x + m] = np.frombuffer(pat, np.uint8)
        else:
            pat = rkgen.iid_text(g, m, table).tobytes()
        t = torch.from_numpy(text).to("cuda:0")
        flags, hs = ctx.paper_search(t, pat, tpb, hashes=True)
        torch.cuda.synchronize()
        nwin = max(n - m + 1, 0)
        assert flags.numel() == nwin
        if nwin == 0:
            continue
        xs = np.arange(nwin, dtype=np.uint64)
        ref_h = oracle.window_hashes(text, m, xs, d=2, q=1 << 32)
        assert np.array_equal(hs.cpu().numpy().astype(np.uint64), ref_h), (trial, m)
        assert np.array_equal(flags.cpu().numpy(), expect_flags(text, pat)), (trial, m)
        pos = ctx.paper_positions(flags).cpu().numpy().astype(np.uint64)
        ro, rp = oracle.search(text, [pat])
        assert pos.tolist() == rp.tolist(), (trial, m)


def test_paper_mode_rejects_hash_collisions(ctx):
    """Windows whose shift-add hash equals the pattern's but whose bytes
    differ ("ac" and "ba" both hash to 2*97 + 99 = 98*2 + 97 = 293) are not
    marked; the paper's sequential loop (the oracle's recompute search with
    d = 2, q = 2^32) agrees."""
    text = np.frombuffer(b"acbaacba" * 1000 + b"ac", np.uint8).copy()
    t = torch.from_numpy(text).to("cuda:0")
    flags, hs = ctx.paper_search(t, b"ac", 256, hashes=True)
    f = flags.cpu().numpy()
    h = hs.cpu().numpy()
    assert (h[0::8] == 293).all() and (h[2::8] == 293).all()  # "ac" and "ba"
    ro, rp = oracle.search_recompute(text, [b"ac"], d=2, q=1 << 32)
    assert np.nonzero(f)[0].tolist() == rp.astype(np.int64).tolist()
    assert f[2::8].sum() == 0


def test_paper_mode_edges(ctx):
    for text, pat in ((b"abc", b"abc"), (b"ab", b"abc"), (b"aaaa", b"a"), (b"\x00\xff" * 300, b"\xff\x00")):
        a = np.frombuffer(text, np.uint8).copy()
        t = torch.from_numpy(a).to("cuda:0")
        flags = ctx.paper_search(t, pat, 64)
        assert np.array_equal(flags.cpu().numpy(), expect_flags(a, pat)), (text[:8], pat)
    # a result array large enough to need more than one grid row of blocks
    g = rkgen.rng(71, 0)
    text = rkgen.iid_text(g, (1 << 22) + 333, rkgen.ACGT)
    pat = text[12345:12352].tobytes()
    t = torch.from_numpy(text).to("cuda:0")
    flags = ctx.paper_search(t, pat, 32)
    pos = ctx.paper_positions(flags).cpu().numpy().astype(np.uint64)
    assert pos.tolist() == oracle.search(text, [pat])[1].tolist()
