"""Pins for the CPU oracle, checked against things other than the oracle itself:
closed forms of the hash, textbook big-integer routines, brute force by
``bytes.find``, exhaustive enumeration, constructed hash collisions and the
planted-occurrence invariants of the generators.  CPU only."""
import itertools
import os

import numpy as np
import pytest

import oracle
import rkgen

Q = (1 << 61) - 1
HERE = os.path.dirname(os.path.abspath(__file__))


def find_all(text: bytes, pat: bytes):
    """Every (overlapping) occurrence via repeated bytes.find."""
    out, i = [], text.find(pat)
    while i >= 0:
        out.append(i)
        i = text.find(pat, i + 1)
    return out


def check_against_find(text: bytes, pats, offsets, positions):
    assert len(offsets) == len(pats) + 1
    assert offsets[0] == 0
    for j, p in enumerate(pats):
        got = positions[int(offsets[j]):int(offsets[j + 1])].tolist()
        assert got == find_all(text, p), (j, p)


# ---------------------------------------------------------------- hash pins
def test_hash_d256_is_big_endian_integer_mod_q():
    """d=256: the polynomial is the window read as a big-endian integer."""
    g = rkgen.rng(90, 0)
    for m in list(range(1, 70)) + [100, 255, 800]:
        w = g.bytes(m)
        assert oracle.hash(w) == int.from_bytes(w, "big") % Q
        if m <= 7:
            assert oracle.hash(w) == int.from_bytes(w, "big")


def test_hash_general_base_is_positional_numeral():
    """Digits 0..d-1 in base d: the hash is the numeral's value mod q,
    computed here by Python's int(str, base) (a textbook conversion)."""
    g = rkgen.rng(90, 1)
    for d in (2, 3, 10, 16, 36):
        for m in (1, 5, 17, 40):
            digits = g.integers(0, d, size=m)
            s = "".join("0123456789abcdefghijklmnopqrstuvwxyz"[x] for x in digits)
            for q in (Q, 1000003, 97):
                assert oracle.hash(bytes(digits.astype(np.uint8)), d, q) == int(s, d) % q


def test_hash_paper_shift_add_example():
    """The paper's hash h = (h << 1) + c: 'ac' and 'ba' give 97*2+99 = 98*2+97 = 293."""
    assert oracle.hash(b"ac", 2, Q) == 293
    assert oracle.hash(b"ba", 2, Q) == 293


def test_pow_256_is_rotation():
    """256^j = 2^(8j mod 61) mod 2^61-1, because 2^61 = 1."""
    for j in range(0, 200):
        assert oracle.pow_mod(256, j, Q) == 1 << ((8 * j) % 61)


def test_golden_window_hashes():
    path = os.path.join(HERE, "golden", "window_hashes.txt")
    n = 0
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        hx, d, q, h = line.split()
        w = bytes.fromhex(hx)
        d, q, h = int(d), int(q), int(h)
        assert oracle.hash(w, d, q) == h
        if d == 256:
            assert h == int.from_bytes(w, "big") % q
        n += 1
    assert n > 70


def test_window_hashes_direct():
    g = rkgen.rng(90, 2)
    text = np.frombuffer(g.bytes(5000), np.uint8)
    for m in (1, 8, 9, 32, 64):
        xs = np.array([0, 1, 4999 - m + 1, 1234, 77], dtype=np.uint64)
        got = oracle.window_hashes(text, m, xs)
        exp = [int.from_bytes(bytes(text[int(x):int(x) + m]), "big") % Q for x in xs]
        assert got.tolist() == exp
    with pytest.raises(ValueError):
        oracle.window_hashes(text, 10, np.array([4991], np.uint64))


def test_constructed_collision_pair():
    """+1 at byte i and -8 at byte i+8 keeps the d=256 hash (2^64 = 8 mod q)."""
    g = rkgen.rng(90, 3)
    for m in (9, 16, 32, 64):
        for _ in range(20):
            w = bytearray(rkgen.LOWER[g.integers(8, 18, size=m)].tobytes())
            i = int(g.integers(0, m - 8))
            w2 = bytearray(w)
            w2[i] += 1
            w2[i + 8] -= 8
            assert oracle.hash(bytes(w)) == oracle.hash(bytes(w2))
            assert int.from_bytes(w, "big") % Q == int.from_bytes(w2, "big") % Q
            assert w != w2


# ---------------------------------------------------------- search pins
def test_exhaustive_binary_alphabet():
    """Every text over {a,b} of length <= 10 against every pattern of length 1..4."""
    pats = [bytes(p) for L in range(1, 5) for p in itertools.product(b"ab", repeat=L)]
    for n in range(0, 11):
        for t in itertools.product(b"ab", repeat=n):
            text = bytes(t)
            off, pos = oracle.search(text, pats)
            check_against_find(text, pats, off, pos)


@pytest.mark.parametrize("alpha", [2, 4, 26, 256])
def test_random_multi_pattern_vs_find(alpha):
    g = rkgen.rng(91, alpha)
    table = {2: np.frombuffer(b"ab", np.uint8), 4: rkgen.ACGT, 26: rkgen.LOWER, 256: rkgen.BYTE256}[alpha]
    for trial in range(12):
        n = int(g.integers(0, 4097))
        text = rkgen.iid_text(g, n, table).tobytes()
        k = int(g.integers(0, 9))
        pats = []
        for j in range(k):
            m = int(g.integers(1, 20))
            if n >= m and g.random() < 0.6:
                o = int(g.integers(0, n - m + 1))
                pats.append(text[o:o + m])
            else:
                pats.append(rkgen.iid_text(g, m, table).tobytes())
        off, pos = oracle.search(text, pats, threads=1 + trial % 4)
        check_against_find(text, pats, off, pos)
        off2, pos2 = oracle.search_recompute(text, pats)
        assert off2.tolist() == off.tolist() and pos2.tolist() == pos.tolist()
        off3, pos3 = oracle.brute(text, pats)
        assert off3.tolist() == off.tolist() and pos3.tolist() == pos.tolist()


def test_small_modulus_forces_verification():
    """With q = 97 most equal hashes are false; the byte check must reject them."""
    g = rkgen.rng(92, 0)
    text = rkgen.iid_text(g, 3000, rkgen.LOWER).tobytes()
    pats = [text[100:108], text[5:6], b"zzzz", text[2990:3000]]
    for q in (97, 2, 3):
        off, pos = oracle.search(text, pats, d=256 % q if 256 % q else 1, q=q)
        check_against_find(text, pats, off, pos)
    off, pos = oracle.search(text, pats, d=2, q=97)
    check_against_find(text, pats, off, pos)


def test_collision_window_not_reported():
    """A window with the pattern's hash but other bytes is not an occurrence."""
    pat = bytearray(b"abcdefghijklmnop")
    col = bytearray(pat)
    col[3] += 1
    col[11] -= 8
    assert oracle.hash(bytes(pat)) == oracle.hash(bytes(col))
    text = b"xx" + bytes(col) + b"yy" + bytes(pat) + bytes(col)
    off, pos = oracle.search(text, [bytes(pat)])
    assert pos.tolist() == [2 + 16 + 2]


def test_edge_cases():
    # first and last window (the sequential pseudo code's bound x < n-m would miss the last)
    off, pos = oracle.search(b"abcab", [b"ab"])
    assert pos.tolist() == [0, 3]
    # m == n, m > n
    off, pos = oracle.search(b"abc", [b"abc", b"abcd"])
    assert off.tolist() == [0, 1, 1] and pos.tolist() == [0]
    # overlaps
    off, pos = oracle.search(b"aaaa", [b"aa", b"a"])
    assert pos.tolist() == [0, 1, 2, 0, 1, 2, 3]
    # bytes 0x00 / 0xFF
    off, pos = oracle.search(b"\x00\xff\x00\xff\x00", [b"\x00\xff", b"\xff\x00\xff"])
    assert pos.tolist() == [0, 2, 1]
    # duplicates each get the full list
    off, pos = oracle.search(b"xyxyx", [b"yx", b"yx"])
    assert off.tolist() == [0, 2, 4] and pos.tolist() == [1, 3, 1, 3]
    # k = 0 and n = 0
    off, pos = oracle.search(b"abc", [])
    assert off.tolist() == [0] and pos.size == 0
    off, pos = oracle.search(b"", [b"a"])
    assert off.tolist() == [0, 0]
    # m = 0 is invalid
    with pytest.raises(ValueError):
        oracle.search(b"abc", [b""])


def test_threads_split_is_seamless():
    """Window ranges split across threads: windows straddling a split are found once."""
    text = (b"ab" * 5000)[:9999]
    pats = [b"ab", b"ba", b"abab", b"b" * 3]
    ref = oracle.search(text, pats, threads=1)
    for t in (2, 3, 7, 16):
        got = oracle.search(text, pats, threads=t)
        assert got[0].tolist() == ref[0].tolist() and got[1].tolist() == ref[1].tolist()
    check_against_find(text, pats, *ref)


# ---------------------------------------------------- planted invariants
def planted_invariants(text: np.ndarray, pat: bytes, plants, offsets, positions):
    pos = positions[int(offsets[0]):int(offsets[1])]
    m = len(pat)
    assert np.all(np.diff(pos.astype(np.int64)) > 0)
    tb = text.tobytes()
    for x in pos.tolist():
        assert tb[x:x + m] == pat
    assert set(int(p) for p in plants) <= set(pos.tolist())
    return pos


def test_config1_planted():
    s = rkgen.config1()
    off, pos = oracle.search(s.text, s.patterns)
    p = planted_invariants(s.text, s.patterns[0], s.manifest["plants"], off, pos)
    assert s.manifest["source"] in p.tolist()
    assert len(p) == 101  # 100 plants + the source window; random extras have p ~ 5e-6
    assert p.tolist() == find_all(s.text.tobytes(), s.patterns[0])


def test_config2_reduced_planted():
    s = rkgen.config2(n=1 << 22, plants=500)
    off, pos = oracle.search(s.text, s.patterns, threads=4)
    p = planted_invariants(s.text, s.patterns[0], s.manifest["plants"], off, pos)
    assert len(p) == 500


def test_config3_reduced_sampled_patterns_found():
    s = rkgen.config3(n=1 << 21, k=64, sampled=32)
    off, pos = oracle.search(s.text, s.patterns, threads=4)
    tb = s.text.tobytes()
    for j, o in enumerate(s.manifest["sampled_offsets"].tolist()):
        assert o in pos[int(off[j]):int(off[j + 1])].tolist()
    check_against_find(tb, s.patterns, off, pos)


def test_search_long_patterns_against_find():
    """Patterns of 65..1024 bytes (longer than any window the GPU scans roll)
    against a bytes.find loop, with overlapping occurrences in a run."""
    g = np.random.default_rng(77)
    text = bytearray(np.frombuffer(g.bytes(20000), np.uint8) % 4 + 65)
    text[5000:7000] = b"A" * 2000
    text = bytes(text)
    pats = [text[o:o + m] for o, m in ((100, 65), (3000, 200), (9000, 1024), (4950, 300))]
    pats += [b"A" * 700, b"A" * 1024, bytes(g.integers(65, 69, size=500, dtype=np.uint8))]
    off, pos = oracle.search(text, pats)
    for j, p in enumerate(pats):
        assert pos[off[j]:off[j + 1]].tolist() == find_all(text, p), j
