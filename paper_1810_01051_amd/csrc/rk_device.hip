// HIP kernels of librk for gfx950 (CDNA4, wave64).
//
// Hot path (Shah & Oza, Sec. 3.1, GPU procedure): every text window gets a
// polynomial hash, the hash is tested against the pattern-hash set and a hit
// is confirmed by comparing bytes.  The paper gives one thread per window and
// recomputes each window's hash from global memory; here a workgroup stages a
// tile of the text (plus a 64-byte halo in front of it) in LDS with coalesced
// 16-byte loads, and each thread rolls the hash over C consecutive windows held
// in registers, so every text byte is read from HBM once.
//
// Window identity: a window is named by its END byte e (bytes e-m+1 .. e).
// Thread t of a tile owns the windows ending at tile bytes [t*C, t*C + C).
//
// Two ways to test a window (same results):
//   exact  : the d=256, q=2^61-1 hash is rolled for every window
//            (H' = 256 H + in - out*256^m mod q, with a lazily reduced 64-bit
//            state) and compared with the set;
//   screen : the paper's shift-and-add hash h' = (h << s) + in mod 2^32 is
//            rolled for every window (s*m >= 32, so bytes older than the window
//            shift out and no out-term is needed); windows whose h is in the
//            set are exact-hashed and looked up in the exact table.
// In both, a candidate window is hashed again from scratch (Horner, canonical
// value), looked up in the exact open-addressing table of its bucket and
// confirmed byte by byte against every pattern chained under that hash.
//
// Hits are compacted with a block-wide prefix sum in ascending window order per
// bucket into a per-tile staging slab; later kernels scan the tile counts,
// compact the slabs and sort stably by pattern id.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rk_internal.h"

// Build-time variants of the scan (the defaults are the measured best on gfx950):
//   RK_PREFETCH  1: a workgroup issues the next tile's loads before processing
//                   the current one; 0: loads, then waits, per tile.
//   RK_MIN_ACC   1: single-target screen ORs matches through a VGPR minimum;
//                0: through per-window wave ballots.
//   RK_WAVES     >0: minimum waves per SIMD requested from the compiler.
#ifndef RK_PREFETCH
#define RK_PREFETCH 1
#endif
#ifndef RK_MIN_ACC
#define RK_MIN_ACC 0
#endif
#ifndef RK_WAVES
#define RK_WAVES 0
#endif

namespace rk {

// ------------------------------------------------------------ arithmetic mod q
// s < 2^63 on input; result < 2^61 + 2^10, congruent to 256*s.
__device__ __forceinline__ uint64_t mul256_lazy(uint64_t s) { return ((s << 8) & kQ) + (s >> 53); }
// s < 2^63 on input; result < 2^61 + 2^34 + ..., congruent to 2^32 * s.
__device__ __forceinline__ uint64_t mul2p32_lazy(uint64_t s) { return ((s << 32) & kQ) + (s >> 29); }
// canonical representative in [0, q) of s < 2^63
__device__ __forceinline__ uint64_t canon(uint64_t s) {
  uint64_t f = (s & kQ) + (s >> 61);  // < 2^61 + 4
  return f >= kQ ? f - kQ : f;
}
// v * 2^r mod q for v < 2^61, 0 <= r < 61 (a rotation of the 61-bit word)
__device__ __forceinline__ uint64_t rot61(uint64_t v, uint32_t r) {
  return ((v << r) & kQ) | (v >> ((61u - r) & 63u));
}

__device__ __forceinline__ uint32_t byte_at(const uint32_t *w, int i) {
  return (w[i >> 2] >> (8 * (i & 3))) & 0xFFu;
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ uint64_t ballot(bool c) { return __builtin_amdgcn_ballot_w64(c); }

// -------------------------------------------------------------- window tests
// Each pass walks the C windows of the calling thread.  The register array w
// holds 64 bytes before the thread's first window end (w[0..15]) followed by
// its C bytes (w[16..]).  ANY=true returns the OR over windows of the wave
// ballot of the test; ANY=false returns the per-thread candidate bit mask.
template <int C>
struct Bits {
  uint32_t b[(C + 31) / 32];
};

// Bit layout of Bits: window i lives in word i/32; inside a word the earliest
// window takes the highest used bit (the flags are shifted in one by one).
template <int C>
__device__ __forceinline__ constexpr int word_windows(int j) {
  return (C - 32 * j) < 32 ? (C - 32 * j) : 32;
}
template <int C>
__device__ __forceinline__ uint32_t bit_of(int i) {
  return 1u << (word_windows<C>(i >> 5) - 1 - (i & 31));
}

// Shifts the flag of window i into the mask.  The empty asm keeps the chain
// sequential; otherwise the OR tree is reassociated and every flag of the
// unrolled loop stays live at once.
template <int C>
__device__ __forceinline__ void put_bit(Bits<C> &bits, uint32_t &acc, int i, bool c) {
  acc = acc + acc + (uint32_t)c;
  __asm__ volatile("" : "+v"(acc));
  if ((i & 31) == 31 || i == C - 1) {
    bits.b[i >> 5] = acc;
    acc = 0;
  }
}

// Register values the compiler must treat as redefined here.  Every test
// variant starts with it so that the byte extractions of the variants are not
// merged and hoisted above the variant switch (which would keep every
// extracted byte of every variant live at once).
template <int NW>
__device__ __forceinline__ void opaque(uint32_t *w) {
#pragma unroll
  for (int j = 0; j < NW; ++j) __asm__ volatile("" : "+v"(w[j]));
}

// The thread's bytes, loaded from the LDS tile by each pass itself so that no
// register copy of them stays live across buckets.
template <int NW>
__device__ __forceinline__ void load_words(uint32_t *w, const uint32_t *tw) {
#pragma unroll
  for (int j = 0; j < NW; ++j) w[j] = tw[j];
  opaque<NW>(w);
}

// OR of the wave ballots, kept as a sequential chain of scalar ORs (a
// reassociated OR tree would keep one SGPR pair per window alive).
__device__ __forceinline__ void any_or(uint64_t &any, uint64_t b) {
  any |= b;
  __asm__ volatile("" : "+s"(any));
}

template <int C, int S, int NT, bool ANY>
__device__ __forceinline__ void pass_list_screen(const uint32_t *tw, uint32_t msk, const uint32_t *tg, uint64_t &any,
                                                 Bits<C> &bits) {
  constexpr int WU = 32 / S - 1;  // bytes needed before the first window end
  uint32_t w[16 + C / 4];
  load_words<16 + C / 4>(w, tw);
  uint32_t h = 0, acc = 0;
#pragma unroll
  for (int j = 64 - WU; j < 64; ++j) h = (h << S) + byte_at(w, j);
  if (RK_MIN_ACC && ANY && NT == 1) {
    // one target: the minimum of h ^ target over the windows is zero iff
    // some window matches; no per-window scalar work
    uint32_t mn = 0xFFFFFFFFu;
#pragma unroll
    for (int i = 0; i < C; ++i) {
      h = (h << S) + byte_at(w, 64 + i);
      const uint32_t v = (S == 8) ? (h & msk) : h;
      mn = min(mn, v ^ tg[0]);
    }
    any_or(any, ballot(mn == 0u));
    return;
  }
#pragma unroll
  for (int i = 0; i < C; ++i) {
    h = (h << S) + byte_at(w, 64 + i);
    const uint32_t v = (S == 8) ? (h & msk) : h;
    if (ANY) {
      uint64_t b = ballot(v == tg[0]);
      if (NT > 1) b |= ballot(v == tg[1]);
      if (NT > 2) b |= ballot(v == tg[2]);
      if (NT > 3) b |= ballot(v == tg[3]);
      any_or(any, b);
    } else {
      bool c = v == tg[0];
      if (NT > 1) c = c || v == tg[1];
      if (NT > 2) c = c || v == tg[2];
      if (NT > 3) c = c || v == tg[3];
      put_bit<C>(bits, acc, i, c);
    }
  }
}

template <int C, int S, bool ANY>
__device__ __forceinline__ void pass_table_screen(const uint32_t *tw, const uint32_t *fp, uint32_t fmask, uint64_t &any,
                                                  Bits<C> &bits) {
  constexpr int WU = 32 / S - 1;
  uint32_t w[16 + C / 4];
  load_words<16 + C / 4>(w, tw);
  uint32_t h = 0, acc = 0;
#pragma unroll
  for (int j = 64 - WU; j < 64; ++j) h = (h << S) + byte_at(w, j);
#pragma unroll
  for (int i = 0; i < C; ++i) {
    h = (h << S) + byte_at(w, 64 + i);
    const uint32_t e = fp[h & fmask];
    const uint32_t f = h >> 16;
    if (ANY) any_or(any, ballot((e & 0xFFFFu) == f) | ballot((e >> 16) == f));
    else put_bit<C>(bits, acc, i, ((e & 0xFFFFu) == f) || ((e >> 16) == f));
  }
}

// Exact rolling hash of the window ending before the first one of this
// thread: Horner over the 64 preceding bytes with the bytes older than the
// window (older than m positions) masked to zero -- leading zero digits do not
// change the polynomial.
__device__ __forceinline__ uint64_t exact_init(const uint32_t *w, uint32_t m) {
  uint64_t s = 0;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int lead = 64 - (int)m - 4 * q;  // bytes of this word that precede the window
    const uint32_t keep = lead <= 0 ? 0xFFFFFFFFu : (lead >= 4 ? 0u : (0xFFFFFFFFu >> (8 * lead)));
    s = mul2p32_lazy(s) + (__builtin_bswap32(w[q]) & keep);
  }
  return s;
}

// One exact rolling step: H(e) = 256 H(e-1) + in - out * 2^r  (r = 8m mod 61).
// s < 2^63 on input, s < 2^62 + 2^11 on output.
__device__ __forceinline__ uint64_t exact_step(uint64_t s, uint32_t in, uint32_t out, uint32_t r) {
  return mul256_lazy(s) + in + (kQ - rot61(out, r));
}

// The same step with the 32-bit halves spelled out and the outgoing term
// specialised on where out * 2^r lands in the 61-bit word (r = 8m mod 61 is
// fixed per group):  OUTK 0: bits r..r+7 in the low word (r <= 24),
// 1: in the high word (32 <= r <= 53), 2: anywhere (general rotation).
//   256 s mod q = ((s << 8) & q) + (s >> 53): the low byte of s << 8 is free
//   for the entering byte; q - v = q ^ v for v <= q.
// Bounds as exact_step: s < 2^63 in, s < 2^62 + 2^11 out.
template <int OUTK>
__device__ __forceinline__ uint64_t exact_step_k(uint64_t s, uint32_t in, uint32_t out, uint32_t r) {
  const uint32_t lo = (uint32_t)s, hi = (uint32_t)(s >> 32);
  const uint32_t alo = (lo << 8) | in;
  const uint32_t ahi = __builtin_amdgcn_alignbit(hi, lo, 24) & 0x1FFFFFFFu;
  uint64_t neg;
  if (OUTK == 0) neg = (0x1FFFFFFFull << 32) | (uint64_t)(uint32_t)~(out << r);
  else if (OUTK == 1) neg = ((uint64_t)(0x1FFFFFFFu ^ (out << (r - 32))) << 32) | 0xFFFFFFFFull;
  else neg = kQ - rot61(out, r);
  return ((((uint64_t)ahi << 32) | alo) + neg) + (hi >> 21);
}

__device__ __forceinline__ int out_kind(uint32_t r) { return r <= 24 ? 0 : ((r >= 32 && r <= 53) ? 1 : 2); }

// Out-stream: the byte leaving window i (the thread's i-th window end) sits m
// bytes before the entering one.  It is read as aligned LDS dwords starting
// o = 4*ceil(m/4) bytes before the thread's first window end and realigned by
// sh = o - m bytes with alignbyte, four windows per dword.
struct OutStream {
  const uint32_t *d;  // LDS, 4-byte aligned
  uint32_t sh;
};

__device__ __forceinline__ OutStream out_stream(const uint8_t *mine, uint32_t m) {
  const uint32_t o = (m + 3u) & ~3u;
  OutStream os;
  os.d = (const uint32_t *)(mine - o);
  os.sh = o - m;
  return os;
}

template <int C, bool ANY, bool TABLE, int NT, int OUTK>
__device__ __forceinline__ void pass_exact(const uint32_t *tw, OutStream os, uint32_t m, uint32_t r, const uint32_t *tg,
                                           const uint32_t *fp, uint32_t fmask, uint64_t &any, Bits<C> &bits) {
  uint32_t w[16 + C / 4];
  load_words<16 + C / 4>(w, tw);
  uint64_t s = exact_init(w, m);
  uint32_t dlo = os.d[0], ow = 0, acc = 0;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    if ((i & 3) == 0) {
      const uint32_t dhi = os.d[(i >> 2) + 1];
      ow = __builtin_amdgcn_alignbyte(dhi, dlo, os.sh);
      dlo = dhi;
    }
    s = exact_step_k<OUTK>(s, byte_at(w, 64 + i), (ow >> (8 * (i & 3))) & 0xFFu, r);
    if (TABLE) {
      const uint32_t h = (uint32_t)canon(s);
      const uint32_t e = fp[h & fmask];
      const uint32_t f = h >> 16;
      if (ANY) any_or(any, ballot((e & 0xFFFFu) == f) | ballot((e >> 16) == f));
      else put_bit<C>(bits, acc, i, ((e & 0xFFFFu) == f) || ((e >> 16) == f));
    } else {
      // lazy state s = H + j*q for j in {0,1,2}; the host lists the low words
      const uint32_t lo = (uint32_t)s;
      if (ANY) {
        uint64_t b = ballot(lo == tg[0]) | ballot(lo == tg[1]);
        if (NT > 2) b |= ballot(lo == tg[2]) | ballot(lo == tg[3]);
        any_or(any, b);
      } else {
        bool c = lo == tg[0] || lo == tg[1];
        if (NT > 2) c = c || lo == tg[2] || lo == tg[3];
        put_bit<C>(bits, acc, i, c);
      }
    }
  }
}

template <int C, bool ANY, bool TABLE, int NT>
__device__ __forceinline__ void pass_exact_r(const uint32_t *tw, OutStream os, uint32_t m, uint32_t r, const uint32_t *tg,
                                             const uint32_t *fp, uint32_t fmask, uint64_t &any, Bits<C> &bits) {
  const int k = out_kind(r);
  if (k == 0) pass_exact<C, ANY, TABLE, NT, 0>(tw, os, m, r, tg, fp, fmask, any, bits);
  else if (k == 1) pass_exact<C, ANY, TABLE, NT, 1>(tw, os, m, r, tg, fp, fmask, any, bits);
  else pass_exact<C, ANY, TABLE, NT, 2>(tw, os, m, r, tg, fp, fmask, any, bits);
}

// kDump: canonical rolling hash of windows x = e - m + 1 with x % stride == 0.
template <int C>
__device__ __forceinline__ void pass_dump(const uint32_t *tw, OutStream os, uint32_t m, uint32_t r, int64_t e0, uint64_t n,
                                          const ScanParams &p) {
  uint32_t w[16 + C / 4];
  load_words<16 + C / 4>(w, tw);
  uint64_t s = exact_init(w, m);
  const int64_t x0 = e0 - (int64_t)m + 1;
  // rem = x0 mod stride for the first window (x0 may be negative)
  const int64_t st = (int64_t)p.dump_stride;
  int64_t rem = x0 % st;
  if (rem < 0) rem += st;
  // slot of the next sampled window at or after x0 (x0 - rem is a multiple of st)
  int64_t slot = (x0 - rem) / st + (rem ? 1 : 0);
  uint32_t dlo = os.d[0], ow = 0;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    if ((i & 3) == 0) {
      const uint32_t dhi = os.d[(i >> 2) + 1];
      ow = __builtin_amdgcn_alignbyte(dhi, dlo, os.sh);
      dlo = dhi;
    }
    s = exact_step(s, byte_at(w, 64 + i), (ow >> (8 * (i & 3))) & 0xFFu, r);
    const int64_t x = x0 + i;
    if (rem == 0) {
      if (x >= 0 && (uint64_t)x + m <= n && (uint64_t)slot < p.dump_cap) p.dump_out[slot] = canon(s);
      ++slot;
    }
    rem = (rem + 1 == st) ? 0 : rem + 1;
  }
}

// Runs the test pass of bucket D over the thread's windows: ANY=true ORs the
// wave ballots into any, ANY=false fills the per-thread candidate mask.
// D.shift holds the screen shift in bits 0-7 and the number of list targets
// (1, or up to 4 padded by repetition) in bits 8-15.
template <int C, bool ANY, int FAM>
__device__ __forceinline__ void run_pass(const BucketDesc &D, const uint32_t *tw, OutStream os, uint32_t r,
                                         const uint32_t *fp, uint64_t &any, Bits<C> &bits) {
  const uint32_t sh = D.shift & 0xFFu;
  if constexpr (FAM == kFamScreen1) {
    if (sh == 1) pass_list_screen<C, 1, 1, ANY>(tw, D.mask, D.tgt, any, bits);
    else if (sh == 2) pass_list_screen<C, 2, 1, ANY>(tw, D.mask, D.tgt, any, bits);
    else if (sh == 4) pass_list_screen<C, 4, 1, ANY>(tw, D.mask, D.tgt, any, bits);
    else pass_list_screen<C, 8, 1, ANY>(tw, D.mask, D.tgt, any, bits);
  } else if constexpr (FAM == kFamScreen) {
    if (D.kind == kListScreen) {
      if ((D.shift >> 8) == 1u) {
        if (sh == 1) pass_list_screen<C, 1, 1, ANY>(tw, D.mask, D.tgt, any, bits);
        else if (sh == 2) pass_list_screen<C, 2, 1, ANY>(tw, D.mask, D.tgt, any, bits);
        else if (sh == 4) pass_list_screen<C, 4, 1, ANY>(tw, D.mask, D.tgt, any, bits);
        else pass_list_screen<C, 8, 1, ANY>(tw, D.mask, D.tgt, any, bits);
      } else {
        if (sh == 1) pass_list_screen<C, 1, 4, ANY>(tw, D.mask, D.tgt, any, bits);
        else if (sh == 2) pass_list_screen<C, 2, 4, ANY>(tw, D.mask, D.tgt, any, bits);
        else if (sh == 4) pass_list_screen<C, 4, 4, ANY>(tw, D.mask, D.tgt, any, bits);
        else pass_list_screen<C, 8, 4, ANY>(tw, D.mask, D.tgt, any, bits);
      }
    } else {
      if (sh == 1) pass_table_screen<C, 1, ANY>(tw, fp, D.fp_mask, any, bits);
      else if (sh == 2) pass_table_screen<C, 2, ANY>(tw, fp, D.fp_mask, any, bits);
      else if (sh == 4) pass_table_screen<C, 4, ANY>(tw, fp, D.fp_mask, any, bits);
      else pass_table_screen<C, 8, ANY>(tw, fp, D.fp_mask, any, bits);
    }
  } else {
    if (D.kind == kListExact) {
      if ((D.shift >> 8) <= 2u) pass_exact_r<C, ANY, false, 2>(tw, os, D.m, r, D.tgt, fp, D.fp_mask, any, bits);
      else pass_exact_r<C, ANY, false, 4>(tw, os, D.m, r, D.tgt, fp, D.fp_mask, any, bits);
    } else {
      pass_exact_r<C, ANY, true, 2>(tw, os, D.m, r, D.tgt, fp, D.fp_mask, any, bits);
    }
  }
}

// ------------------------------------------------------- block-level helpers
template <int WG>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *wsum, uint32_t &total) {
  constexpr int NW = WG / 64;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += y;
  }
  __syncthreads();
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint32_t before = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const uint32_t s = wsum[i];
    before += (uint32_t)i < wave ? s : 0u;
    tot += s;
  }
  total = tot;
  return before + x - v;
}

// Exact hash (canonical) of m bytes at p (LDS), Horner.
__device__ __forceinline__ uint64_t horner_exact(const uint8_t *p, uint32_t m) {
  uint64_t s = 0;
  for (uint32_t j = 0; j < m; ++j) s = mul256_lazy(s) + p[j];
  return canon(s);
}

// Shift-add hash of the span = 32/s bytes ending at *end (the value the scan's
// screen pass held for that window end), masked as the group's hash is.
__device__ __forceinline__ uint32_t screen_key(const uint8_t *end, uint32_t shift, uint32_t mask) {
  const uint32_t span = 32u / shift;
  uint32_t h = 0;
  for (uint32_t j = span; j-- > 0;) h = (h << shift) + end[-(int)j];
  return h & mask;
}

// Run of entries (first | count << 16) stored under key, or kNoLink.
__device__ __forceinline__ uint32_t key_lookup(const uint8_t *img, const BucketDesc &D, uint64_t key) {
  const uint64_t *keys = (const uint64_t *)(img + D.ht_off);
  const uint32_t *runs = (const uint32_t *)(img + D.ht_off + 8u * (D.ht_mask + 1u));
  uint32_t slot = ht_slot(key, D.ht_mask);
  for (uint32_t probe = 0; probe <= D.ht_mask; ++probe) {
    const uint64_t k = keys[slot];
    if (k == key) return runs[slot];
    if (k == kEmptyKey) return kNoLink;
    slot = (slot + 1u) & D.ht_mask;
  }
  return kNoLink;
}

__device__ __forceinline__ bool bytes_equal(const uint8_t *a, const uint8_t *b, uint32_t m) {
  for (uint32_t j = 0; j < m; ++j)
    if (a[j] != b[j]) return false;
  return true;
}

// Walks the run of entries found for the candidate window ending at *end
// (global end index e) and calls hit(entry) for every pattern that occurs
// there: the window of the entry's length must start inside the text, have
// the entry's exact hash and equal bytes.  Entries of a run are sorted by
// length, so one backward pass accumulates the exact hash of every suffix:
// S_m = sum_{j<m} T[e-j] * 256^j = hash of the m-byte window ending at e.
template <typename F>
__device__ __forceinline__ void verify_run(const uint8_t *img, const BucketDesc &D, uint32_t run, const uint8_t *end,
                                           int64_t e, F &&hit) {
  if (run == kNoLink) return;
  const Entry *ent = (const Entry *)(img + D.ent_off);
  const uint32_t first = run & 0xFFFFu, cnt = run >> 16;
  uint64_t S = 0;   // lazy: < 2^62
  uint32_t j = 0;   // bytes accumulated
  uint32_t r = 0;   // 8j mod 61
  for (uint32_t t = first; t < first + cnt; ++t) {
    const uint32_t m = ent[t].off_m >> 24;
    if (e - (int64_t)m + 1 < 0) continue;  // window would start before the text
    for (; j < m; ++j) {
      S += rot61((uint64_t)end[-(int)j], r);
      S = (S & kQ) + (S >> 61);
      r = (r + 8u >= 61u) ? r + 8u - 61u : r + 8u;
    }
    if (canon(S) != ent[t].hx) continue;
    if (bytes_equal(end - (m - 1), img + D.pat_off + (ent[t].off_m & 0xFFFFFFu), m)) hit(ent[t]);
  }
}

// ------------------------------------------------------------ the scan kernel
//
// LDS: [tile: kFront + W + 16][cand: kCandCap u32][misc: 64 u32][image: img_cap]
template <int WG, int C, int FAM>
#if RK_WAVES > 0
__global__ __launch_bounds__(WG, RK_WAVES) void scan_kernel(ScanParams p) {
#else
__global__ __launch_bounds__(WG) void scan_kernel(ScanParams p) {
#endif
  constexpr uint32_t W = WG * C;
  constexpr uint32_t TILE_LDS = (kFront + W + 16 + 15) & ~15u;
  constexpr uint32_t NCH = (kFront + W) / 16;  // 16-byte chunks loaded per tile
  constexpr uint32_t LOADS = (NCH + WG - 1) / WG;
  constexpr int NB = (C + 31) / 32;
  extern __shared__ __align__(16) uint8_t lds[];
  uint8_t *tile = lds;
  uint32_t *cand = (uint32_t *)(lds + TILE_LDS);
  uint32_t *misc = cand + kCandCap;  // [0,16) scan sums, [16,48) any flags, [48] queue
  uint8_t *img = (uint8_t *)(misc + 64);

  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t cur_inst = kNoLink;
  uint64_t static_item = blockIdx.x;
  uint32_t flag_parity = 0;
  const uint64_t nitems = p.nitems_dev ? min(p.nitems, (uint64_t)*p.nitems_dev) : p.nitems;

  // Next work item (uniform across the workgroup).  With a queue, thread 0
  // pops and the value is read back after the barrier that follows.
  auto pop = [&]() -> uint64_t {
    if (p.queue) {
      __syncthreads();
      if (tid == 0) misc[48] = atomicAdd(p.queue, 1u);
      __syncthreads();
      return misc[48];
    }
    const uint64_t it = static_item;
    static_item += gridDim.x;
    return it;
  };
  struct Item {
    uint64_t gt;
    uint32_t inst;
    const uint8_t *text;
    uint64_t n;
    int64_t tstart;
  };
  auto locate = [&](uint64_t item) -> Item {
    Item it;
    it.gt = p.items ? p.items[item] : item;
    uint32_t lo = 0, hi = p.ninst;  // instance owning global tile gt
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (p.inst[mid].tile_base <= it.gt) lo = mid;
      else hi = mid;
    }
    it.inst = lo;
    it.text = p.inst[lo].text;
    it.n = p.inst[lo].n;
    it.tstart = (int64_t)((it.gt - p.inst[lo].tile_base) * W);
    return it;
  };
  // text bytes [tstart - kFront, tstart + W) in aligned 16-byte chunks
  uint4 v[LOADS];
  auto issue_loads = [&](const Item &it) {
#pragma unroll
    for (uint32_t u = 0; u < LOADS; ++u) {
      const uint32_t q = tid + u * WG;
      const int64_t g = it.tstart - (int64_t)kFront + 16 * (int64_t)q;
      v[u] = make_uint4(0, 0, 0, 0);
      if (q < NCH && g >= 0 && (uint64_t)g < it.n) v[u] = *(const uint4 *)(it.text + g);
    }
  };

  uint64_t item = pop();
  Item cur;
  if (item < nitems) {
    cur = locate(item);
    if (RK_PREFETCH) issue_loads(cur);
  }
  while (item < nitems) {
    const uint64_t next = pop();  // ends with a barrier when a queue is used
    if (!RK_PREFETCH) issue_loads(cur);
    __syncthreads();  // previous tile finished with tile / cand / image
    if (cur.inst != cur_inst) {
      const uint4 *src = (const uint4 *)(p.blob + p.inst[cur.inst].img_off);
      uint4 *dst = (uint4 *)img;
      const uint32_t nq = p.inst[cur.inst].img_bytes / 16u;
      for (uint32_t q = tid; q < nq; q += WG) dst[q] = src[q];
      cur_inst = cur.inst;
    }
#pragma unroll
    for (uint32_t u = 0; u < LOADS; ++u) {
      const uint32_t q = tid + u * WG;
      if (q < NCH) *(uint4 *)(tile + 16 * q) = v[u];
    }
    __syncthreads();
    // the next tile's loads are in flight while this one is processed
    Item nx;
    if (next < nitems) {
      nx = locate(next);
      if (RK_PREFETCH) issue_loads(nx);
    }
    const uint64_t gt = cur.gt;
    const uint64_t n = cur.n;
    const int64_t tstart = cur.tstart;

    // this thread's bytes: 64 before its first window end, then C
    const uint32_t *tw = (const uint32_t *)(tile + kFront + tid * C - 64);
    const uint8_t *mine = tile + kFront + tid * C;  // LDS byte of my first window end
    const int64_t e0 = tstart + (int64_t)(tid * C); // global end index of my first window

    const ImageHeader *H = (const ImageHeader *)img;
    const uint32_t nb = uni(H->nbuckets);
    uint32_t tile_hits = 0;
    uint64_t *slab = nullptr;
    if (p.out) slab = p.direct ? (p.out + p.tile_offsets[gt]) : (p.out + gt * (uint64_t)p.slab_cap);
    const uint32_t cap = p.direct ? 0xFFFFFFFFu : p.slab_cap;

    for (uint32_t b = 0; b < nb; ++b) {
      const BucketDesc *dp = (const BucketDesc *)(img + sizeof(ImageHeader) + 64u * b);
      BucketDesc D;
      D.m = uni(dp->m);
      D.kind = uni(dp->kind);
      D.shift = uni(dp->shift);
      D.mask = uni(dp->mask);
#pragma unroll
      for (int j = 0; j < 4; ++j) D.tgt[j] = uni(dp->tgt[j]);
      D.fp_off = uni(dp->fp_off);
      D.fp_mask = uni(dp->fp_mask);
      D.ht_off = uni(dp->ht_off);
      D.ht_mask = uni(dp->ht_mask);
      D.ent_off = uni(dp->ent_off);
      D.max_m = uni(dp->max_m);
      D.pat_off = uni(dp->pat_off);
      D.npat = uni(dp->npat);
      const uint32_t m = D.m;
      const uint32_t r = (8u * m) % 61u;
      const uint32_t *fp = (const uint32_t *)(img + D.fp_off);
      const OutStream os = out_stream(mine, m);

      if constexpr (FAM == kFamExact) {
        if (D.kind == kDump) {
          pass_dump<C>(tw, os, m, r, e0, n, p);
          continue;
        }
      }

      // ---- pass 1: wave-level "any candidate" over every window
      uint64_t any = 0;
      Bits<C> nob;
      run_pass<C, true, FAM>(D, tw, os, r, fp, any, nob);
      uint32_t *flags = misc + 16 + 16 * flag_parity;
      flag_parity ^= 1u;
      if (lane == 0) flags[wave] = any != 0;
      __syncthreads();
      uint32_t blk_any = 0;
#pragma unroll
      for (int i = 0; i < WG / 64; ++i) blk_any |= flags[i];
      if (!blk_any) continue;

      // ---- pass 2 (only when some window of the tile passed): per-thread masks
      Bits<C> bits;
#pragma unroll
      for (int j = 0; j < NB; ++j) bits.b[j] = 0;
      uint64_t dummy = 0;
      run_pass<C, false, FAM>(D, tw, os, r, fp, dummy, bits);
      // only windows with m-1 <= e <= n-1 exist
      const bool edge = tstart < (int64_t)m - 1 || (uint64_t)(tstart + W) > n;
      if (edge) {
        // my windows i are valid for ilo <= i < ihi
        const int64_t lo64 = (int64_t)m - 1 - e0, hi64 = (int64_t)n - e0;
        const int ilo = (int)(lo64 < 0 ? 0 : (lo64 > C ? C : lo64));
        const int ihi = (int)(hi64 < 0 ? 0 : (hi64 > C ? C : hi64));
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const int nw = word_windows<C>(j);
          int a = ilo - 32 * j, b2 = ihi - 32 * j;
          a = a < 0 ? 0 : (a > nw ? nw : a);
          b2 = b2 < 0 ? 0 : (b2 > nw ? nw : b2);
          // local window k sits at bit nw-1-k: keep bits [nw-b2, nw-a)
          const uint32_t below_hi = (nw - a) >= 32 ? 0xFFFFFFFFu : ((1u << (nw - a)) - 1u);
          const uint32_t below_lo = (nw - b2) >= 32 ? 0xFFFFFFFFu : ((1u << (nw - b2)) - 1u);
          bits.b[j] &= (b2 > a) ? (below_hi & ~below_lo) : 0u;
        }
      }
      uint32_t cnt = 0;
#pragma unroll
      for (int j = 0; j < NB; ++j) cnt += __builtin_popcount(bits.b[j]);
      uint32_t ncand;
      const uint32_t cbase = block_excl_scan<WG>(cnt, misc, ncand);

      for (uint32_t r0 = 0; r0 < ncand; r0 += kCandCap) {
        __syncthreads();  // cand list free
        if (cnt) {
          uint32_t idx = cbase;
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            uint32_t bb = bits.b[j];
            while (bb) {
              const uint32_t hb = 31u - __builtin_clz(bb);  // highest bit = earliest window
              const uint32_t i = 32u * j + (uint32_t)word_windows<C>(j) - 1u - hb;
              bb &= ~(1u << hb);
              if (idx >= r0 && idx < r0 + kCandCap) cand[idx - r0] = tid * C + i;
              ++idx;
            }
          }
        }
        __syncthreads();
        const uint32_t nc = min(kCandCap, ncand - r0);
        for (uint32_t i0 = 0; i0 < nc; i0 += WG) {
          const uint32_t ci = i0 + tid;
          uint32_t run = kNoLink, nh = 0;
          const uint8_t *end = nullptr;
          int64_t e = 0;
          const bool screen = D.kind == kListScreen || D.kind == kTableScreen;
          if (ci < nc) {
            const uint32_t e_rel = cand[ci];
            end = tile + kFront + e_rel;
            e = tstart + (int64_t)e_rel;
            const uint64_t key = screen ? (uint64_t)screen_key(end, D.shift & 0xFFu, D.mask)
                                        : horner_exact(end - (m - 1), m);
            run = key_lookup(img, D, key);
            verify_run(img, D, run, end, e, [&](const Entry &) { ++nh; });
          }
          uint32_t nht;
          const uint32_t hb = block_excl_scan<WG>(nh, misc, nht);
          if (nh) {
            uint32_t o = tile_hits + hb;
            verify_run(img, D, run, end, e, [&](const Entry &en) {
              const uint64_t x = (uint64_t)(e - (int64_t)(en.off_m >> 24) + 1);
              if (o < cap) slab[o] = ((uint64_t)en.pid << kPosBits) | x;
              ++o;
            });
          }
          tile_hits += nht;
        }
      }
    }

    if (tid == 0 && !p.direct) {
      p.tile_counts[gt] = tile_hits;
      if (tile_hits) atomicAdd(p.total, (unsigned long long)tile_hits);
      if (tile_hits > p.slab_cap) {
        const uint32_t o = atomicAdd(p.ovf_count, 1u);
        p.ovf_list[o] = gt;
      }
    }
    item = next;
    cur = nx;
  }
}

// ---------------------------------------------------------- prefix sums (u64)
// Exclusive scan of u32 counts into u64 offsets, three kernels:
// per-block sums, a single-block scan of those sums, per-block local scans.
constexpr int kScanWG = 256;
constexpr int kScanPer = 16;
constexpr int kScanBlock = kScanWG * kScanPer;  // items per block

__global__ __launch_bounds__(kScanWG) void scan_block_sums(const uint32_t *in, uint64_t n, uint64_t *bsum) {
  __shared__ uint64_t red[kScanWG / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const uint64_t i = base + (uint64_t)j * kScanWG + threadIdx.x;
    if (i < n) s += in[i];
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int i = 0; i < kScanWG / 64; ++i) t += red[i];
    bsum[blockIdx.x] = t;
  }
}

// Single block: exclusive scan of bsum[0..nb) in place; bsum[nb] = total;
// also copies the total to *total_out if non-null.
__global__ __launch_bounds__(1024) void scan_sums_single(uint64_t *bsum, uint64_t nb, uint64_t *total_out) {
  __shared__ uint64_t wsum[16];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (uint64_t base = 0; base < nb; base += 1024) {
    const uint64_t i = base + threadIdx.x;
    const uint64_t v = i < nb ? bsum[i] : 0;
    uint64_t x = v;
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t y = __shfl_up(x, d, 64);
      if (lane >= (uint32_t)d) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    uint64_t before = carry, tot = 0;
    for (int k = 0; k < 16; ++k) {
      before += (uint32_t)k < wave ? wsum[k] : 0;
      tot += wsum[k];
    }
    if (i < nb) bsum[i] = before + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bsum[nb] = carry;
    if (total_out) *total_out = carry;
  }
}

__global__ __launch_bounds__(kScanWG) void scan_local(const uint32_t *in, uint64_t n, const uint64_t *bsum,
                                                      uint64_t *out) {
  __shared__ uint64_t wsum[kScanWG / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // each thread owns kScanPer consecutive items
  uint32_t v[kScanPer];
  uint64_t s = 0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const uint64_t i = base + (uint64_t)threadIdx.x * kScanPer + j;
    v[j] = i < n ? in[i] : 0u;
    s += v[j];
  }
  uint64_t x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = __shfl_up(x, d, 64);
    if (lane >= (uint32_t)d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint64_t before = bsum[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanWG / 64; ++k) before += (uint32_t)k < wave ? wsum[k] : 0;
  uint64_t run = before + x - s;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const uint64_t i = base + (uint64_t)threadIdx.x * kScanPer + j;
    if (i < n) out[i] = run;
    run += v[j];
  }
}

// ------------------------------------------------------------ slab compaction
// One wave per tile: copy the tile's staged hits to their final offset
// (tiles that overflowed their slab are rescanned instead).
__global__ __launch_bounds__(256) void compact_slabs(const uint32_t *counts, const uint64_t *offs, uint64_t ntiles,
                                                     const uint64_t *slabs, uint32_t slab_cap, uint64_t *out) {
  const uint64_t t = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const uint32_t c = counts[t];
  if (c == 0 || c > slab_cap) return;
  const uint64_t *src = slabs + t * (uint64_t)slab_cap;
  uint64_t *dst = out + offs[t];
  for (uint32_t i = threadIdx.x & 63; i < c; i += 64) dst[i] = src[i];
}

// -------------------------------------------------- stable radix by pattern id
// Records are pid << 40 | x.  One 8-bit digit of the pid per pass; a block is
// one wave walking its kRadixBlock records 64 at a time in order, so ranks are
// stable.
constexpr int kRadixBlock = 1024;

__global__ __launch_bounds__(64) void radix_hist(const uint64_t *in, uint64_t n, uint32_t shift, uint32_t *ghist,
                                                 uint64_t nblk) {
  __shared__ uint32_t h[256];
  for (int i = threadIdx.x; i < 256; i += 64) h[i] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kRadixBlock;
  for (int j = 0; j < kRadixBlock; j += 64) {
    const uint64_t i = base + j + threadIdx.x;
    if (i < n) atomicAdd(&h[(in[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < 256; d += 64) ghist[(uint64_t)d * nblk + blockIdx.x] = h[d];
}

__global__ __launch_bounds__(64) void radix_scatter(const uint64_t *in, uint64_t n, uint32_t shift,
                                                    const uint64_t *goff, uint64_t nblk, uint64_t *out) {
  __shared__ uint64_t run[256];
  for (int d = threadIdx.x; d < 256; d += 64) run[d] = goff[(uint64_t)d * nblk + blockIdx.x];
  __syncthreads();
  const uint32_t lane = threadIdx.x;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  const uint64_t base = (uint64_t)blockIdx.x * kRadixBlock;
  for (int j = 0; j < kRadixBlock; j += 64) {
    const uint64_t i = base + j + lane;
    const bool valid = i < n;
    const uint64_t rec = valid ? in[i] : 0;
    const uint32_t dg = (uint32_t)(rec >> shift) & 255u;
    // lanes holding the same digit
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t ones = ballot(valid && ((dg >> bit) & 1u));
      peers &= ((dg >> bit) & 1u) ? ones : ~ones;
    }
    const uint32_t rank = __builtin_popcountll(peers & lt_mask);
    const uint64_t dst = run[dg] + rank;
    __syncthreads();
    if (valid) {
      out[dst] = rec;
      // the highest lane of each digit group advances the cursor
      if ((peers >> lane) == 1ull) run[dg] += __builtin_popcountll(peers);
    }
    __syncthreads();
  }
}

// offsets[j] = first index of pid j in the sorted records; offsets[k] = n.
__global__ void pid_offsets(const uint64_t *sorted, uint64_t n, uint32_t k, uint64_t *offsets) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j > k) return;
  if (j == k) {
    offsets[k] = n;
    return;
  }
  uint64_t lo = 0, hi = n;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if ((sorted[mid] >> kPosBits) < j) lo = mid + 1;
    else hi = mid;
  }
  offsets[j] = lo;
}

__global__ void strip_positions(const uint64_t *rec, uint64_t n, uint64_t *pos) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) pos[i] = rec[i] & kPosMask;
}

__global__ void single_offsets(uint64_t *offsets, uint64_t total) {
  if (threadIdx.x == 0) {
    offsets[0] = 0;
    offsets[1] = total;
  }
}

// ------------------------------------------------------------- window hashes
__global__ void window_hashes_kernel(const uint8_t *text, uint64_t n, uint32_t m, const uint64_t *xs, uint64_t cnt,
                                     uint64_t *out) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const uint64_t x = xs[i];
  if (m == 0 || x > n || n - x < m) {
    out[i] = ~0ull;
    return;
  }
  uint64_t s = 0;
  for (uint32_t j = 0; j < m; ++j) s = mul256_lazy(s) + text[x + j];
  out[i] = canon(s);
}

// ------------------------------------------------------------------ launchers
template <int WG, int C, int FAM>
static hipError_t launch_scan_t(const ScanParams &p, uint32_t grid, uint32_t lds_bytes, hipStream_t s) {
  // the dynamic LDS limit was raised by prepare_scan_kernels() at context creation
  hipLaunchKernelGGL((scan_kernel<WG, C, FAM>), dim3(grid), dim3(WG), lds_bytes, s, p);
  return hipGetLastError();
}

template <int WG, int C, int FAM>
static hipError_t occ_t(uint32_t lds_bytes, int *blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void *)scan_kernel<WG, C, FAM>, WG, lds_bytes);
}

template <int FAM>
static hipError_t launch_fam(int cfg, const ScanParams &p, uint32_t grid, uint32_t lds_bytes, hipStream_t s) {
  switch (cfg) {
    case 0: return launch_scan_t<256, 68, FAM>(p, grid, lds_bytes, s);
    case 1: return launch_scan_t<256, 132, FAM>(p, grid, lds_bytes, s);
    case 2: return launch_scan_t<512, 68, FAM>(p, grid, lds_bytes, s);
    case 3: return launch_scan_t<256, 36, FAM>(p, grid, lds_bytes, s);
    default: return hipErrorInvalidValue;
  }
}

template <int FAM>
static hipError_t occ_fam(int cfg, uint32_t lds_bytes, int *blocks) {
  switch (cfg) {
    case 0: return occ_t<256, 68, FAM>(lds_bytes, blocks);
    case 1: return occ_t<256, 132, FAM>(lds_bytes, blocks);
    case 2: return occ_t<512, 68, FAM>(lds_bytes, blocks);
    case 3: return occ_t<256, 36, FAM>(lds_bytes, blocks);
    default: return hipErrorInvalidValue;
  }
}

hipError_t scan_occupancy(int cfg, int fam, uint32_t lds_bytes, int *blocks) {
  switch (fam) {
    case kFamScreen1: return occ_fam<kFamScreen1>(cfg, lds_bytes, blocks);
    case kFamScreen: return occ_fam<kFamScreen>(cfg, lds_bytes, blocks);
    case kFamExact: return occ_fam<kFamExact>(cfg, lds_bytes, blocks);
    default: return hipErrorInvalidValue;
  }
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t words, uint32_t v) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < words) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t words, uint32_t v, hipStream_t s) {
  if (words == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((uint32_t)((words + 255) / 256)), dim3(256), 0, s, p, words, v);
  return hipGetLastError();
}

uint32_t scan_lds_bytes(int cfg, uint32_t img_cap) {
  const TileCfg c = kTileCfgs[cfg];
  const uint32_t W = c.wg * c.c;
  const uint32_t tile = (kFront + W + 16 + 15) & ~15u;
  return tile + kCandCap * 4 + 64 * 4 + img_cap;
}

hipError_t launch_scan(int cfg, int fam, const ScanParams &p, uint32_t grid, uint32_t lds_bytes, hipStream_t s) {
  switch (fam) {
    case kFamScreen1: return launch_fam<kFamScreen1>(cfg, p, grid, lds_bytes, s);
    case kFamScreen: return launch_fam<kFamScreen>(cfg, p, grid, lds_bytes, s);
    case kFamExact: return launch_fam<kFamExact>(cfg, p, grid, lds_bytes, s);
    default: return hipErrorInvalidValue;
  }
}

// exclusive scan of n u32 counts into u64 offsets; tmp holds scan_tmp_words(n)
// u64; *total_dev (optional) receives the sum.
uint64_t scan_tmp_words(uint64_t n) { return (n + kScanBlock - 1) / kScanBlock + 2; }

hipError_t launch_exclusive_scan(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *tmp, uint64_t *total_dev,
                                 hipStream_t s) {
  const uint64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb > 0) hipLaunchKernelGGL(scan_block_sums, dim3((uint32_t)nb), dim3(kScanWG), 0, s, in, n, tmp);
  hipLaunchKernelGGL(scan_sums_single, dim3(1), dim3(1024), 0, s, tmp, nb, total_dev);
  if (nb > 0) hipLaunchKernelGGL(scan_local, dim3((uint32_t)nb), dim3(kScanWG), 0, s, in, n, tmp, out);
  return hipGetLastError();
}

hipError_t launch_compact(const uint32_t *counts, const uint64_t *offs, uint64_t ntiles, const uint64_t *slabs,
                          uint32_t slab_cap, uint64_t *out, hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  hipLaunchKernelGGL(compact_slabs, dim3((uint32_t)((ntiles + 3) / 4)), dim3(256), 0, s, counts, offs, ntiles, slabs,
                     slab_cap, out);
  return hipGetLastError();
}

uint64_t radix_blocks(uint64_t n) { return (n + kRadixBlock - 1) / kRadixBlock; }

// Stable sort of n records by pid (bits 40.. of each record), npass digits of
// 8 bits; ping-pongs between a and b; returns the buffer holding the result.
hipError_t launch_radix(uint64_t *a, uint64_t *b, uint64_t n, uint32_t npass, uint32_t *ghist, uint64_t *goff,
                        uint64_t *tmp, uint64_t **result, hipStream_t s) {
  const uint64_t nblk = radix_blocks(n);
  uint64_t *src = a, *dst = b;
  for (uint32_t ps = 0; ps < npass && n > 0; ++ps) {
    const uint32_t shift = kPosBits + 8 * ps;
    hipLaunchKernelGGL(radix_hist, dim3((uint32_t)nblk), dim3(64), 0, s, src, n, shift, ghist, nblk);
    hipError_t e = launch_exclusive_scan(ghist, 256 * nblk, goff, tmp, nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(radix_scatter, dim3((uint32_t)nblk), dim3(64), 0, s, src, n, shift, goff, nblk, dst);
    uint64_t *t = src;
    src = dst;
    dst = t;
  }
  *result = src;
  return hipGetLastError();
}

hipError_t launch_pid_offsets(const uint64_t *sorted, uint64_t n, uint32_t k, uint64_t *offsets, hipStream_t s) {
  const uint64_t th = (uint64_t)k + 1;
  hipLaunchKernelGGL(pid_offsets, dim3((uint32_t)((th + 255) / 256)), dim3(256), 0, s, sorted, n, k, offsets);
  return hipGetLastError();
}

hipError_t launch_strip(const uint64_t *rec, uint64_t n, uint64_t *pos, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(strip_positions, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s, rec, n, pos);
  return hipGetLastError();
}

hipError_t launch_single_offsets(uint64_t *offsets, uint64_t total, hipStream_t s) {
  hipLaunchKernelGGL(single_offsets, dim3(1), dim3(64), 0, s, offsets, total);
  return hipGetLastError();
}

hipError_t launch_window_hashes(const uint8_t *text, uint64_t n, uint32_t m, const uint64_t *xs, uint64_t cnt,
                                uint64_t *out, hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(window_hashes_kernel, dim3((uint32_t)((cnt + 255) / 256)), dim3(256), 0, s, text, n, m, xs, cnt,
                     out);
  return hipGetLastError();
}

// Raises the dynamic LDS limit of every scan kernel once, outside any stream
// capture (a graph capture must not run first-time setup calls).
template <int FAM>
static void prepare_fam() {
  (void)hipFuncSetAttribute((const void *)scan_kernel<256, 68, FAM>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  (void)hipFuncSetAttribute((const void *)scan_kernel<256, 132, FAM>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  (void)hipFuncSetAttribute((const void *)scan_kernel<512, 68, FAM>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
  (void)hipFuncSetAttribute((const void *)scan_kernel<256, 36, FAM>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            160 * 1024);
}

void prepare_scan_kernels() {
  prepare_fam<kFamScreen1>();
  prepare_fam<kFamScreen>();
  prepare_fam<kFamExact>();
}

}  // namespace rk

namespace rk {

// ----------------------------------------------------- stream-read roofline
// Reads every 16-byte block of data[0..n) once (the scan's load width, fully
// coalesced, grid-stride) and folds it into one word per workgroup so that
// nothing is optimised away: the read-bandwidth ceiling the scan is held to.
__global__ __launch_bounds__(256) void stream_read_kernel(const uint4 *data, uint64_t nblk, uint32_t *out) {
  uint32_t acc = 0;
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  for (; i + 3 * stride < nblk; i += 4 * stride) {
    const uint4 a = data[i], b = data[i + stride], c = data[i + 2 * stride], d = data[i + 3 * stride];
    acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
  }
  for (; i < nblk; i += stride) {
    const uint4 a = data[i];
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  for (int d = 32; d >= 1; d >>= 1) acc ^= __shfl_xor(acc, d, 64);
  __shared__ uint32_t red[4];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = red[0] ^ red[1] ^ red[2] ^ red[3];
}

hipError_t launch_stream_read(const void *data, uint64_t n, uint32_t *out, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(stream_read_kernel, dim3(grid), dim3(256), 0, s, (const uint4 *)data, n / 16, out);
  return hipGetLastError();
}

}  // namespace rk

namespace rk {

// ------------------------------------------------------- segmented copy
// dst_k[0..len_k) = src[src_off_k .. src_off_k + len_k) for every segment;
// the server uses it to give each request a contiguous copy of its patterns'
// hit lists out of a merged step.  Segments are at most 65536 entries long.
__global__ __launch_bounds__(256) void segment_copy_kernel(const uint64_t *src, const CopySeg *segs, uint32_t nseg) {
  for (uint32_t s = blockIdx.x; s < nseg; s += gridDim.x) {
    const CopySeg g = segs[s];
    for (uint64_t i = threadIdx.x; i < g.len; i += 256) g.dst[i] = src[g.src_off + i];
  }
}

hipError_t launch_segment_copy(const uint64_t *src, const CopySeg *segs, uint32_t nseg, hipStream_t s) {
  if (nseg == 0) return hipSuccess;
  const uint32_t grid = nseg < 4096 ? nseg : 4096;
  hipLaunchKernelGGL(segment_copy_kernel, dim3(grid), dim3(256), 0, s, src, segs, nseg);
  return hipGetLastError();
}

}  // namespace rk
