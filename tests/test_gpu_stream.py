"""Streamed searches of texts in host memory and in files (rk_search_host,
rk_search_file) against the oracle: occurrences planted across piece
boundaries, short and long patterns, both modes, piece sizes down to the
minimum, and the degenerate texts."""
import numpy as np
import pytest

import oracle
import rkgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

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


def planted_text(seed, n, pats, piece):
    g = rkgen.rng(90, seed)
    text = rkgen.iid_text(g, n, rkgen.ACGT)
    mmax = max(len(p) for p in pats)
    L = ((piece + 15) // 16 * 16) - (mmax - 1)
    for p in pats:
        m = len(p)
        for b in range(L, n, L):
            for d in (-m, -m + 1, -1, 0, 1):
                x = b + d
                if 0 <= x <= n - m:
                    text[x:x + m] = np.frombuffer(p, np.uint8)
    return text


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("piece", [1 << 16, (1 << 18) + 5, 1 << 20])
def test_host_text_pieces(ctx, rk, mode, piece):
    g = rkgen.rng(91, piece)
    pats = [rkgen.ACGT[g.integers(0, 4, size=m)].tobytes() for m in (1, 7, 32, 64, 65, 300, 1024)]
    n = 6 * (1 << 20) + 123
    text = planted_text(piece, n, pats, piece)
    pats.append(text[5000:5016].tobytes())
    plan = rk.Plan(ctx, pats, mode)
    off, pos = plan.search_host(text, piece)
    plan.close()
    ro, rp = oracle.search(text, pats, threads=4)
    assert int(ro[-1]) > 100
    assert off.tolist() == ro.tolist()
    assert pos.tolist() == rp.tolist()


@pytest.mark.parametrize("mode", MODES)
def test_file_text(ctx, rk, mode, tmp_path):
    g = rkgen.rng(92, 0)
    pats = [b"ACGTACGTAC", rkgen.ACGT[g.integers(0, 4, size=200)].tobytes(), b"A"]
    text = planted_text(7, 3 * (1 << 20) + 17, pats, 1 << 18)
    path = tmp_path / "text.bin"
    path.write_bytes(text.tobytes())
    plan = rk.Plan(ctx, pats, mode)
    off, pos = plan.search_host(str(path), 1 << 18)
    plan.close()
    ro, rp = oracle.search(text, pats, threads=4)
    assert off.tolist() == ro.tolist() and pos.tolist() == rp.tolist()


def test_stream_edges(ctx, rk):
    plan = rk.Plan(ctx, [b"abc", b"b"], "screen")
    for text in (b"", b"ab", b"abc", b"xabcabc" * 20000):
        off, pos = plan.search_host(np.frombuffer(text, np.uint8), 1 << 16)
        ro, rp = oracle.search(text, [b"abc", b"b"])
        assert off.tolist() == ro.tolist() and pos.tolist() == rp.tolist(), len(text)
    with pytest.raises(rk._lib.RkError) as e:
        plan.search_host(np.zeros(10, np.uint8), 1000)
    assert e.value.status == rk._lib.RK_EINVAL
    plan.close()
