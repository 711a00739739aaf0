"""Seeded synthetic inputs for the Rabin-Karp search (texts, pattern sets,
planted occurrences, batches of uneven instances, request streams).

This package holds no hashing or matching arithmetic: it only draws bytes.
Both the CPU oracle side and the GPU side take their inputs from here.

Every stream is ``numpy.random.Generator(PCG64(SeedSequence(ROOT_SEED,
spawn_key=(cfg, sub))))`` so a (config, sub-stream) pair always yields the same
bytes.  The workloads stand in for the paper's randomly generated DNA files
(Sec. 3.3) and extend them to the multi-pattern, batched and serving cases.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ROOT_SEED = 0x181001051
ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)
LOWER = np.arange(ord("a"), ord("z") + 1, dtype=np.uint8)
BYTE256 = np.arange(256, dtype=np.uint8)
_GEN_CHUNK = 1 << 26  # bytes drawn per call; part of the recipe (fixes the stream layout)


def rng(cfg: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(ROOT_SEED, spawn_key=(cfg, sub))))


def iid_text(g: np.random.Generator, n: int, alphabet: np.ndarray) -> np.ndarray:
    """n bytes drawn i.i.d. uniformly from ``alphabet`` (drawn in fixed-size chunks)."""
    out = np.empty(n, dtype=np.uint8)
    a = len(alphabet)
    for s in range(0, n, _GEN_CHUNK):
        e = min(n, s + _GEN_CHUNK)
        if a == 256:
            out[s:e] = np.frombuffer(g.bytes(e - s), dtype=np.uint8)
        elif a & (a - 1) == 0:  # power-of-two alphabet: low bits of raw random bytes
            table = bytes(int(alphabet[i & (a - 1)]) for i in range(256))
            out[s:e] = np.frombuffer(g.bytes(e - s).translate(table), dtype=np.uint8)
        else:
            out[s:e] = alphabet[g.integers(0, a, size=e - s, dtype=np.uint8)]
    return out


def nonoverlapping_offsets(g: np.random.Generator, n: int, m: int, count: int,
                           forbid: list[int] | tuple = ()) -> np.ndarray:
    """``count`` sorted window starts in [0, n-m] whose windows [o, o+m) do not
    overlap each other nor the windows starting at ``forbid`` (rejection)."""
    if count == 0:
        return np.zeros(0, dtype=np.int64)
    if count * m + len(forbid) * m > n // 2:
        raise ValueError("too many plants for the text length")
    chosen: list[int] = []
    blocked = sorted(int(f) for f in forbid)
    while len(chosen) < count:
        cand = g.integers(0, n - m + 1, size=2 * (count - len(chosen)) + 8, dtype=np.int64)
        for c in cand.tolist():
            i = np.searchsorted(blocked, c)
            ok = True
            if i < len(blocked) and blocked[i] - c < m:
                ok = False
            if i > 0 and c - blocked[i - 1] < m:
                ok = False
            if ok:
                blocked.insert(int(i), c)
                chosen.append(c)
                if len(chosen) == count:
                    break
    return np.array(sorted(chosen), dtype=np.int64)


@dataclass
class Search:
    """One search instance: a text, a pattern list and what was planted."""
    text: np.ndarray
    patterns: list
    manifest: dict = field(default_factory=dict)


def config1(n: int = 1 << 20, m: int = 8, plants: int = 100) -> Search:
    """Single short pattern: n bytes U{'a'..'z'}; the pattern is copied from a
    random text offset and planted ``plants`` more times (non-overlapping)."""
    g = rng(1, 0)
    text = iid_text(g, n, LOWER)
    src = int(g.integers(0, n - m + 1))
    pat = bytes(text[src:src + m])
    offs = nonoverlapping_offsets(g, n, m, plants, forbid=[src])
    pv = np.frombuffer(pat, dtype=np.uint8)
    for o in offs.tolist():
        text[o:o + m] = pv
    return Search(text, [pat], {"source": src, "plants": offs})


def config2(n: int = 1 << 32, m: int = 32, plants: int = 10_000) -> Search:
    """Single long pattern over DNA: n bytes U{A,C,G,T}; one random ACGT pattern
    planted at ``plants`` non-overlapping seeded offsets."""
    g = rng(2, 0)
    text = iid_text(g, n, ACGT)
    gp = rng(2, 1)
    pv = ACGT[gp.integers(0, 4, size=m)]
    offs = nonoverlapping_offsets(gp, n, m, plants)
    for o in offs.tolist():
        text[o:o + m] = pv
    return Search(text, [pv.tobytes()], {"plants": offs})


def zipf_vocab(g: np.random.Generator, words: int = 50_000, lmin: int = 3, lmax: int = 12):
    lens = g.integers(lmin, lmax + 1, size=words)
    letters = LOWER[g.integers(0, 26, size=int(lens.sum()), dtype=np.uint8)]
    return lens.astype(np.int64), letters


def zipf_text(g: np.random.Generator, n: int, lens: np.ndarray, letters: np.ndarray,
              s: float = 1.1, chunk_words: int = 1 << 22) -> np.ndarray:
    """Words drawn from a finite Zipf law P(rank r) ~ r^-s (word i has rank i+1),
    joined by single spaces and cut to exactly n bytes."""
    W = len(lens)
    p = np.arange(1, W + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    # vocabulary blob: each word followed by one space
    wl = lens + 1
    wstart = np.zeros(W, dtype=np.int64)
    wstart[1:] = np.cumsum(wl)[:-1]
    blob = np.empty(int(wl.sum()), dtype=np.uint8)
    blob[:] = ord(" ")
    src_off = np.zeros(W, dtype=np.int64)
    src_off[1:] = np.cumsum(lens)[:-1]
    idx = np.repeat(wstart - src_off, lens) + np.arange(int(lens.sum()), dtype=np.int64)
    blob[idx] = letters
    del idx
    out = np.empty(n, dtype=np.uint8)
    filled = 0
    while filled < n:
        u = g.random(chunk_words)
        r = np.searchsorted(cdf, u, side="right")
        r = np.minimum(r, W - 1)
        L = wl[r]
        tot = int(L.sum())
        take = min(tot, n - filled)
        ends = np.cumsum(L)
        starts = ends - L
        gidx = np.repeat(wstart[r] - starts, L) + np.arange(tot, dtype=np.int64)
        out[filled:filled + take] = blob[gidx[:take]]
        filled += take
    return out


def config3(n: int = 1 << 30, k: int = 1024, m: int = 16, sampled: int = 512) -> Search:
    """Multi-pattern over word text: Zipf(1.1) words from a 50,000-word vocabulary
    (lengths U{3..12} over 'a'..'z'); ``sampled`` patterns are text[o:o+m] for
    uniform o, the other k-sampled are uniform random 'a'..'z' strings."""
    g = rng(3, 0)
    lens, letters = zipf_vocab(g)
    text = zipf_text(rng(3, 1), n, lens, letters)
    gp = rng(3, 2)
    pats = []
    offs = gp.integers(0, n - m + 1, size=sampled)
    for o in offs.tolist():
        pats.append(bytes(text[o:o + m]))
    rnd = LOWER[gp.integers(0, 26, size=(k - sampled, m), dtype=np.uint8)]
    for row in rnd:
        pats.append(row.tobytes())
    return Search(text, pats, {"sampled_offsets": offs})


def config4(count: int = 4096, lmin: int = 4096, lmax: int = 16 << 20, kmax: int = 32,
            mmin: int = 4, mmax: int = 64, copies: int = 8) -> list[Search]:
    """Uneven batch: text lengths log-uniform in [lmin, lmax], alphabet size
    uniform in {4, 26, 256}, 1..kmax patterns of length U{mmin..mmax}; pattern j
    is planted ``copies`` times iff j is even (later plants may overwrite)."""
    g = rng(4, 0)
    out = []
    alph = {4: ACGT, 26: LOWER, 256: BYTE256}
    for i in range(count):
        L = int(math.exp(g.uniform(math.log(lmin), math.log(lmax))))
        a = int(g.choice([4, 26, 256]))
        gi = rng(4, 1 + i)
        text = iid_text(gi, L, alph[a])
        k = int(g.integers(1, kmax + 1))
        pats = []
        planted = {}
        for j in range(k):
            m = int(g.integers(mmin, mmax + 1))
            pv = alph[a][gi.integers(0, a, size=m)]
            pats.append(pv.tobytes())
            if j % 2 == 0 and m <= L:
                offs = gi.integers(0, L - m + 1, size=copies)
                for o in offs.tolist():
                    text[o:o + m] = pv
                planted[j] = offs
        out.append(Search(text, pats, {"alphabet": a, "planted": planted}))
    return out


def config5_corpus(index: int, n: int = 1 << 30, device="cuda:0", chunk_words: int = 1 << 22):
    """Serving corpus ``index``: the config-3 word text recipe with its own
    vocabulary and rank stream, drawn on the GPU with torch (seeded Philox) so
    that 64 corpora of 1 GiB are ready in seconds.  Returns a uint8 tensor."""
    import torch
    g = rng(5, 2 * index)
    lens, letters = zipf_vocab(g)
    W = len(lens)
    p = np.arange(1, W + 1, dtype=np.float64) ** (-1.1)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    wl = lens + 1
    wstart = np.zeros(W, dtype=np.int64)
    wstart[1:] = np.cumsum(wl)[:-1]
    blob = np.full(int(wl.sum()), ord(" "), dtype=np.uint8)
    src_off = np.zeros(W, dtype=np.int64)
    src_off[1:] = np.cumsum(lens)[:-1]
    blob[np.repeat(wstart - src_off, lens) + np.arange(int(lens.sum()), dtype=np.int64)] = letters
    dev = torch.device(device)
    cdf_t = torch.from_numpy(cdf).to(dev)
    wl_t = torch.from_numpy(wl).to(dev)
    ws_t = torch.from_numpy(wstart).to(dev)
    blob_t = torch.from_numpy(blob).to(dev)
    tg = torch.Generator(device=dev)
    tg.manual_seed(int(rng(5, 2 * index + 1).integers(0, 2**62)))
    out = torch.empty(n, dtype=torch.uint8, device=dev)
    filled = 0
    while filled < n:
        u = torch.rand(chunk_words, generator=tg, device=dev, dtype=torch.float64)
        r = torch.searchsorted(cdf_t, u, right=True).clamp_(max=W - 1)
        L = wl_t[r]
        ends = torch.cumsum(L, 0)
        tot = int(ends[-1])
        take = min(tot, n - filled)
        word = torch.repeat_interleave(torch.arange(chunk_words, device=dev), L)[:take]
        within = torch.arange(take, device=dev) - (ends - L)[word]
        out[filled:filled + take] = blob_t[ws_t[r[word]] + within]
        filled += take
    return out


def config5_request_specs(rate: float, duration: float, corpus_len: int, corpora: int = 64, kmax: int = 256,
                          mmin: int = 4, mmax: int = 64, seed_sub: int = 0):
    """Like config5_requests, but a sampled pattern is returned as its
    (offset, length) in the target corpus, so that a caller holding the
    corpora on the device can gather all sampled bytes at once.  Each request
    is (t_arrival, corpus, [bytes | (offset, length), ...])."""
    g = rng(5, 1000 + seed_sub)
    t = 0.0
    out = []
    while True:
        t += float(g.exponential(1.0 / rate))
        if t >= duration:
            break
        c = int(g.integers(0, corpora))
        k = int(g.integers(1, kmax + 1))
        pats = []
        for j in range(k):
            m = int(g.integers(mmin, mmax + 1))
            if j % 2 == 0:
                pats.append((int(g.integers(0, corpus_len - m + 1)), m))
            else:
                pats.append(LOWER[g.integers(0, 26, size=m, dtype=np.uint8)].tobytes())
        out.append((t, c, pats))
    return out


@dataclass
class Request:
    t_arrival: float
    corpus: int
    patterns: list


def config5_requests(rate: float, duration: float, corpora: int = 64, kmax: int = 256,
                     mmin: int = 4, mmax: int = 64, sample_text=None, seed_sub: int = 0):
    """Open-loop Poisson arrivals at ``rate`` req/s for ``duration`` seconds.
    Each request targets a uniform corpus and carries U{1..kmax} patterns of
    length U{mmin..mmax}; half are sampled from the target corpus (through
    ``sample_text(corpus, g, m)`` returning bytes), half random 'a'..'z'."""
    g = rng(5, 1000 + seed_sub)
    t = 0.0
    reqs = []
    while True:
        t += float(g.exponential(1.0 / rate))
        if t >= duration:
            break
        c = int(g.integers(0, corpora))
        k = int(g.integers(1, kmax + 1))
        pats = []
        for j in range(k):
            m = int(g.integers(mmin, mmax + 1))
            if j % 2 == 0 and sample_text is not None:
                pats.append(bytes(sample_text(c, g, m)))
            else:
                pats.append(LOWER[g.integers(0, 26, size=m, dtype=np.uint8)].tobytes())
        reqs.append(Request(t, c, pats))
    return reqs
