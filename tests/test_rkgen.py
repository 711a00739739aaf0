"""The seeded input generators: determinism and the stated shapes of each
workload (CPU only, reduced sizes)."""
import math

import numpy as np

import rkgen


def test_streams_are_deterministic():
    a = rkgen.config1()
    b = rkgen.config1()
    assert np.array_equal(a.text, b.text) and a.patterns == b.patterns
    assert a.manifest["source"] == b.manifest["source"]


def test_config1_shape():
    s = rkgen.config1()
    assert s.text.size == 1 << 20 and len(s.patterns) == 1 and len(s.patterns[0]) == 8
    assert set(np.unique(s.text).tolist()) <= set(range(ord("a"), ord("z") + 1))
    plants = s.manifest["plants"]
    assert len(plants) == 100 and np.all(np.diff(plants) >= 8)
    assert all(abs(int(p) - s.manifest["source"]) >= 8 for p in plants)


def test_config2_shape_reduced():
    s = rkgen.config2(n=1 << 20, plants=50)
    assert set(np.unique(s.text).tolist()) <= set(b"ACGT")
    counts = np.bincount(s.text, minlength=256)[[65, 67, 71, 84]]
    assert counts.min() > 0.24 * s.text.size and counts.max() < 0.26 * s.text.size
    assert len(s.patterns[0]) == 32 and np.all(np.diff(s.manifest["plants"]) >= 32)


def test_config3_zipf_text():
    s = rkgen.config3(n=1 << 20, k=64, sampled=32)
    t = s.text.tobytes()
    words = t.split(b" ")[1:-1]
    assert all(3 <= len(w) <= 12 for w in words)
    # finite Zipf(1.1) over 50,000 words: the most frequent word is about 13.9% of tokens
    top = max(np.unique(np.array(words, dtype=object), return_counts=True)[1]) / len(words)
    assert 0.12 < top < 0.16
    assert len(s.patterns) == 64 and all(len(p) == 16 for p in s.patterns)
    assert all(s.patterns[j] == t[o:o + 16] for j, o in enumerate(s.manifest["sampled_offsets"].tolist()))


def test_config4_shapes():
    insts = rkgen.config4(count=40, lmax=1 << 16)
    for s in insts:
        assert 4096 <= len(s.text) <= 1 << 16
        assert s.manifest["alphabet"] in (4, 26, 256)
        assert 1 <= len(s.patterns) <= 32 and all(4 <= len(p) <= 64 for p in s.patterns)
        assert set(s.manifest["planted"]) <= set(range(0, len(s.patterns), 2))
    # log-uniform mean over [4 KiB, 16 MiB] (the realized total the full config gives)
    mean = (16 * 2**20 - 4096) / math.log(4096)
    assert 1.8 * 2**20 < mean < 2.0 * 2**20


def test_config5_specs_match_callback_stream():
    n = 1 << 16
    text = rkgen.iid_text(rkgen.rng(77, 0), n, rkgen.LOWER)

    def sample(c, g, m):
        o = int(g.integers(0, n - m + 1))
        return text[o:o + m].tobytes()

    reqs = rkgen.config5_requests(500.0, 0.2, corpora=4, sample_text=sample)
    specs = rkgen.config5_request_specs(500.0, 0.2, n, corpora=4)
    assert len(reqs) == len(specs) and len(reqs) > 50
    for r, (t, c, pats) in zip(reqs, specs):
        assert r.t_arrival == t and r.corpus == c and len(r.patterns) == len(pats)
        for p, q in zip(r.patterns, pats):
            if isinstance(q, tuple):
                assert p == text[q[0]:q[0] + q[1]].tobytes()
            else:
                assert p == q
