"""The autotuner (rk_autotune) checked against the oracle: every candidate
geometry's result, for one pattern per length and for every batch bucket
shape, has the hit count and digest of the oracle's search of the same text
and patterns (both rebuilt here from the recipe rk.h states)."""
import json

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

M64 = (1 << 64) - 1
CLASS_LO = (1, 4, 8, 16, 32)
CLASS_HI = (3, 7, 15, 31, 64)
CLASS_K = (1, 4, 32, 256)


def tuner_text(n):
    """Knuth's MMIX linear congruential sequence, byte i = "ACGT"[x_i >> 62]."""
    out = np.empty(n, np.uint8)
    x = 0x181001051
    acgt = b"ACGT"
    for i in range(n):
        x = (x * 6364136223846793005 + 1442695040888963407) & M64
        out[i] = acgt[x >> 62]
    return out


def bucket_patterns(text, nb, mc, kc):
    lo, hi = CLASS_LO[mc], CLASS_HI[mc]
    pats = []
    for j in range(CLASS_K[kc]):
        m = lo + j % (hi - lo + 1)
        o = (nb // 3 + 7919 * j) % (nb - m + 1)
        p = text[o:o + m].tobytes()
        pats.append(p[::-1] if j & 1 else p)
    return pats


def digest(off, pos):
    v = np.concatenate([off.astype(np.uint64), pos.astype(np.uint64)])
    w = (2 * np.arange(v.size, dtype=np.uint64) + 1)
    with np.errstate(over="ignore"):
        return int(np.sum(v * w, dtype=np.uint64))


def test_autotune_candidates_match_oracle(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1810_01051_amd as rk
    n = 1 << 20
    lengths = [4, 7, 32, 64]
    ctx = rk.Context(0)
    path = str(tmp_path / "tune.json")
    ctx.autotune(n, lengths, path)
    table = json.load(open(path))
    text = tuner_text(n)
    singles = {}
    for row in table["timings"]:
        m = row["m"]
        if m not in singles:
            ro, rp = oracle.search(text, [text[n // 3:n // 3 + m].tobytes()])
            singles[m] = (int(ro[-1]), digest(ro, rp))
        assert (row["hits"], row["digest"]) == singles[m], row
    assert len(table["timings"]) == len(lengths) * 2 * 4
    seen = {}
    for row in table["bucket_timings"]:
        key = (row["mclass"], row["kclass"])
        if key not in seen:
            nb = row["n"]
            pats = bucket_patterns(text, nb, *key)
            assert len(pats) == row["k"]
            ro, rp = oracle.search(text[:nb], pats, threads=4)
            seen[key] = (int(ro[-1]), digest(ro, rp))
        assert (row["hits"], row["digest"]) == seen[key], row
    assert len(table["bucket_timings"]) == 2 * 5 * 4 * 4
    # the context holds the table's choices, and a reload gives the same
    for b in table["buckets"]:
        mode = "exact" if b["bmode"] == 1 else "screen"
        assert ctx.autotune_bucket_choice(mode, b["mclass"], b["kclass"]) == b["cfg"]
    ctx2 = rk.Context(0)
    ctx2.autotune_load(path)
    for b in table["buckets"]:
        mode = "exact" if b["bmode"] == 1 else "screen"
        assert ctx2.autotune_bucket_choice(mode, b["mclass"], b["kclass"]) == b["cfg"]
    for c in table["choice"]:
        mode = "exact" if c["mode"] == 1 else "screen"
        assert ctx2.autotune_choice(mode, c["m"]) == c["cfg"]
    ctx2.close()
    ctx.close()
