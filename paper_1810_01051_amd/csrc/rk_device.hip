// HIP kernels of librk for gfx950 that follow the scan: prefix sums of the
// per-tile hit counts, slab compaction, the stable radix sort by pattern id,
// per-pattern offsets, direct window hashes and the stream-read roofline probe;
// plus the dispatch of the scan kernels (rk_scan.h, instantiated per family and
// geometry in the rk_scan_*.hip units).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rk_dev.h"
#include "rk_internal.h"
#include "rk_runtime.h"

namespace rk {

// ---------------------------------------------------------- prefix sums (u64)
// Exclusive scan of u32 counts into u64 offsets: per-block sums, then
// per-block local scans that start from the sum of the blocks before them,
// which up to kScanWG blocks add up themselves and beyond that a single-block
// scan of the sums (scan_sums_single) hands them.  Every block is kScanWG
// threads: a scan of one step is not held back until a whole CU is free while
// another step's scan fills the chip.
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
__global__ __launch_bounds__(kScanWG) void scan_sums_single(uint64_t *bsum, uint64_t nb, uint64_t *total_out) {
  __shared__ uint64_t wsum[kScanWG / 64];
  __shared__ uint64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (uint64_t base = 0; base < nb; base += kScanWG) {
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
    for (int k = 0; k < kScanWG / 64; ++k) {
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

// RAW: bsum holds the blocks' own sums (at most kScanWG blocks), each block
// adds those before it, and the last one writes the total (bsum[nb], and
// *total_out if non-null); else bsum is already scanned.
template <bool RAW>
__global__ __launch_bounds__(kScanWG) void scan_local(const uint32_t *in, uint64_t n, uint64_t *bsum, uint64_t nb,
                                                      uint64_t *out, uint64_t *total_out) {
  __shared__ uint64_t wsum[kScanWG / 64];
  __shared__ uint64_t pre[kScanWG / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kScanBlock;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (RAW) {
    uint64_t p = threadIdx.x < blockIdx.x ? bsum[threadIdx.x] : 0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) p += __shfl_xor(p, d, 64);
    if (lane == 0) pre[wave] = p;
  }
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
  uint64_t before = 0;
  if (RAW) {
#pragma unroll
    for (int k = 0; k < kScanWG / 64; ++k) before += pre[k];
  } else {
    before = bsum[blockIdx.x];
  }
#pragma unroll
  for (int k = 0; k < kScanWG / 64; ++k) before += (uint32_t)k < wave ? wsum[k] : 0;
  uint64_t run = before + x - s;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    const uint64_t i = base + (uint64_t)threadIdx.x * kScanPer + j;
    if (i < n) out[i] = run;
    run += v[j];
  }
  if (RAW && blockIdx.x == nb - 1 && threadIdx.x == kScanWG - 1) {
    bsum[nb] = run;
    if (total_out) *total_out = run;
  }
}

// ------------------------------------------------------------ slab compaction
// Copy every tile's staged hits to their final offset (tiles that overflowed
// their slab are rescanned instead).  offsets1 (a single pattern's offsets,
// else null) gets {0, total} from the first thread.
//
// compact_slabs: one wave per tile.
__global__ __launch_bounds__(256) void compact_slabs(const uint32_t *counts, const uint64_t *offs, uint64_t ntiles,
                                                     const uint64_t *slabs, uint32_t slab_cap, uint64_t *out,
                                                     uint64_t *offsets1, uint64_t total) {
  if (offsets1 && blockIdx.x == 0 && threadIdx.x == 0) {
    offsets1[0] = 0;
    offsets1[1] = total;
  }
  const uint64_t t = (uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= ntiles) return;
  const uint32_t c = counts[t];
  if (c == 0 || c > slab_cap) return;
  const uint64_t *src = slabs + t * (uint64_t)slab_cap;
  uint64_t *dst = out + offs[t];
  for (uint32_t i = threadIdx.x & 63; i < c; i += 64) dst[i] = src[i];
}

// compact_sparse (fewer hits than tiles): a wave takes 64 tiles, a lane
// each.  A lane copies its tile itself when it holds at most kLaneCopy
// records; the wave copies the larger ones, one after the other.
constexpr uint32_t kLaneCopy = 8;

__global__ __launch_bounds__(256) void compact_sparse(const uint32_t *counts, const uint64_t *offs, uint64_t ntiles,
                                                      const uint64_t *slabs, uint32_t slab_cap, uint64_t *out,
                                                      uint64_t *offsets1, uint64_t total) {
  if (offsets1 && blockIdx.x == 0 && threadIdx.x == 0) {
    offsets1[0] = 0;
    offsets1[1] = total;
  }
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t t0 = ((uint64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 64, t = t0 + lane;
  const uint32_t c = t < ntiles ? counts[t] : 0u;
  const bool ok = c != 0 && c <= slab_cap;
  const uint64_t o = ok ? offs[t] : 0;
  if (ok && c <= kLaneCopy) {
    const uint64_t *src = slabs + t * (uint64_t)slab_cap;
    uint64_t r[kLaneCopy];
#pragma unroll
    for (uint32_t i = 0; i < kLaneCopy; ++i)
      if (i < c) r[i] = src[i];
#pragma unroll
    for (uint32_t i = 0; i < kLaneCopy; ++i)
      if (i < c) out[o + i] = r[i];
  }
  uint64_t big = __ballot(ok && c > kLaneCopy);
  while (big) {
    const uint32_t l = (uint32_t)__builtin_ctzll(big);
    big &= big - 1;
    const uint32_t cl = __shfl(c, (int)l, 64);
    const uint64_t ol = __shfl(o, (int)l, 64);
    const uint64_t *src = slabs + (t0 + l) * (uint64_t)slab_cap;
    for (uint32_t i = lane; i < cl; i += 64) out[ol + i] = src[i];
  }
}

// -------------------------------------------------- stable radix by pattern id
// Records are pid << 40 | x.  One DB-bit digit of the pid per pass (8 bits,
// or 9..11 when a single pass covers every pid); a block is one wave walking
// its BLK records in order, so ranks are stable.  Each lane loads kRadixR
// records before it handles any, so that a wave keeps kRadixR * 64 loads in
// flight instead of one round trip per 64 records.
constexpr int kRadixBlock = 1024;        // records per block, 8-bit digits
constexpr int kRadixBlock11 = 8192;      // records per block, 9..11-bit digits (at most 2048 digits per block)
constexpr int kRadixR = 16;              // records per lane in flight

// BM: the histogram is block-major (block b's ND counts contiguous, the
// one-pass sorts); else digit-major (the 8-bit passes, scanned as one array).
template <int DB, int BLK, bool BM>
__global__ __launch_bounds__(64) void radix_hist(const uint64_t *in, uint64_t n, uint32_t shift, uint32_t *ghist,
                                                 uint64_t nblk) {
  constexpr uint32_t ND = 1u << DB;
  static_assert(BLK % (64 * kRadixR) == 0, "block is whole rounds");
  __shared__ uint32_t h[ND];
  for (uint32_t i = threadIdx.x; i < ND; i += 64) h[i] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * BLK;
  for (int j = 0; j < BLK; j += 64 * kRadixR) {
    uint64_t rec[kRadixR];
#pragma unroll
    for (int u = 0; u < kRadixR; ++u) {
      const uint64_t i = base + j + u * 64 + threadIdx.x;
      rec[u] = i < n ? in[i] : ~0ull;
    }
#pragma unroll
    for (int u = 0; u < kRadixR; ++u)
      if (rec[u] != ~0ull) atomicAdd(&h[(rec[u] >> shift) & (ND - 1u)], 1u);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < ND; d += 64)
    ghist[BM ? (uint64_t)blockIdx.x * ND + d : (uint64_t)d * nblk + blockIdx.x] = h[d];
}

// STRIP: the pass is the last one, and writes each record's position only
// (the final positions array) instead of the record.  Ranks within 64
// records: every lane ORs its bit into the LDS mask of its digit, reads the
// mask back (the lanes holding that digit) and counts the lower ones; the
// highest lane of each digit advances the digit's cursor and clears the
// mask.  The block is one wave, whose LDS operations take effect in issue
// order, so no barrier is needed between those steps.
template <int DB, int BLK, bool STRIP, bool BM>
__global__ __launch_bounds__(64) void radix_scatter(const uint64_t *in, uint64_t n, uint32_t shift,
                                                    const uint64_t *goff, uint64_t nblk, uint64_t *out) {
  constexpr uint32_t ND = 1u << DB;
  __shared__ uint64_t run[ND];
  __shared__ unsigned long long grp[ND];
  for (uint32_t d = threadIdx.x; d < ND; d += 64) {
    run[d] = goff[BM ? (uint64_t)blockIdx.x * ND + d : (uint64_t)d * nblk + blockIdx.x];
    grp[d] = 0;
  }
  __syncthreads();
  const uint32_t lane = threadIdx.x;
  const uint64_t me = 1ull << lane, lt_mask = me - 1ull;
  // rounds of 64 * kRadixR records; the next round's loads are issued before
  // the current one is ranked, all unconditional (indices clamped to the
  // block's last record, the lanes past it skipped when ranking)
  const uint64_t base = (uint64_t)blockIdx.x * BLK, end = min(base + BLK, n);
  auto load_round = [&](uint64_t j, uint64_t (&r)[kRadixR]) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < kRadixR; ++u) r[u] = in[min(j + (uint64_t)u * 64u + lane, end - 1)];
  };
  uint64_t cur[kRadixR];
  load_round(base, cur);
  for (uint64_t j = base;; j += 64u * kRadixR) {
    // (a block of one round has no next one: 8-bit passes)
    const bool more = BLK > 64 * kRadixR && j + 64u * kRadixR < end;
    uint64_t nxt[kRadixR];
    if constexpr (BLK > 64 * kRadixR) load_round(more ? j + 64u * kRadixR : j, nxt);
#pragma unroll
    for (int u = 0; u < kRadixR; ++u) {
      if (j + (uint64_t)u * 64u + lane >= end) continue;
      const uint64_t rec = cur[u];
      const uint32_t dg = (uint32_t)(rec >> shift) & (ND - 1u);
      atomicOr(&grp[dg], (unsigned long long)me);
      const uint64_t peers = grp[dg];
      const uint64_t at = run[dg];
      out[at + __builtin_popcountll(peers & lt_mask)] = STRIP ? (rec & kPosMask) : rec;
      if ((peers >> lane) == 1ull) {
        run[dg] = at + __builtin_popcountll(peers);
        grp[dg] = 0;
      }
    }
    if (!more) break;
    if constexpr (BLK > 64 * kRadixR) {
#pragma unroll
      for (int u = 0; u < kRadixR; ++u) cur[u] = nxt[u];
    }
  }
}

// ------------------------------- one radix pass reading the staging slabs
// For dense hits the compaction is skipped: the records of a part's tiles
// are read where the count pass left them, tile by tile in tile order (the
// order the compaction would have produced), a block taking G consecutive
// tiles.  Tile t's counts[t] records are its slab (slabs + (t - tile0) * S)
// when they fit, else those of the collect's rescan, written at tile_off[t]
// of the direct buffer.
__device__ __forceinline__ const uint64_t *tile_records(const TileSrc &src, uint64_t t, uint32_t &c) {
  c = __builtin_amdgcn_readfirstlane(src.counts[t]);
  return c <= src.S ? src.slabs + (t - src.tile0) * src.S : src.direct + src.tile_off[t];
}

// Four waves per block, wave w taking the block's tiles w, w + 4, ...
template <int DB>
__global__ __launch_bounds__(256) void radix_hist_tiles(TileSrc src, uint32_t *ghist, uint64_t nblk) {
  constexpr uint32_t ND = 1u << DB;
  __shared__ uint32_t h[ND];
  for (uint32_t i = threadIdx.x; i < ND; i += 256) h[i] = 0;
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t t0 = src.tile0 + (uint64_t)blockIdx.x * src.G;
  const uint64_t t1 = min(t0 + src.G, src.tile0 + src.ntiles);
  for (uint64_t t = t0 + w; t < t1; t += 4) {
    uint32_t c;
    const uint64_t *in = tile_records(src, t, c);
    for (uint32_t j = 0; j < c; j += 64 * kRadixR) {
      uint64_t rec[kRadixR];
#pragma unroll
      for (int u = 0; u < kRadixR; ++u) {
        const uint32_t i = j + u * 64 + lane;
        rec[u] = i < c ? in[i] : ~0ull;
      }
#pragma unroll
      for (int u = 0; u < kRadixR; ++u)
        if (rec[u] != ~0ull) atomicAdd(&h[(rec[u] >> kPosBits) & (ND - 1u)], 1u);
    }
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < ND; d += 256) ghist[(src.blk0 + blockIdx.x) * ND + d] = h[d];
}

// Positions of the records to their final place (the last and only pass),
// ranked as in radix_scatter.  The block's tiles are one stream of rounds of
// 64 * kRadixR records.  A round's loads are unconditional (indices clamped
// to the tile's last record; the lanes past it are skipped when ranking), so
// that the compiler can count them, and the next round's loads are issued
// before the current round is ranked: a wave then waits for its loads once
// per two rounds' latency instead of draining before every round.
__device__ __forceinline__ void tiles_load_round(const uint64_t *in, uint32_t j, uint32_t c, uint64_t (&r)[kRadixR]) {
#pragma unroll
  for (int u = 0; u < kRadixR; ++u) r[u] = in[min(j + (uint32_t)u * 64u + threadIdx.x, c - 1u)];
}

template <int DB>
__global__ __launch_bounds__(64) void radix_scatter_tiles(TileSrc src, const uint64_t *goff, uint64_t nblk,
                                                          uint64_t *out) {
  constexpr uint32_t ND = 1u << DB;
  __shared__ uint64_t run[ND];
  __shared__ unsigned long long grp[ND];
  const uint64_t b = src.blk0 + blockIdx.x;
  for (uint32_t d = threadIdx.x; d < ND; d += 64) {
    run[d] = goff[b * ND + d];
    grp[d] = 0;
  }
  __syncthreads();
  const uint32_t lane = threadIdx.x;
  const uint64_t me = 1ull << lane, lt_mask = me - 1ull;
  const uint64_t t0 = src.tile0 + (uint64_t)blockIdx.x * src.G;
  const uint64_t t1 = min(t0 + src.G, src.tile0 + src.ntiles);
  // the first tile holding records (the round is (t, j): records j.. of tile t)
  uint64_t t = t0;
  uint32_t c = 0, j = 0;
  const uint64_t *in = nullptr;
  for (; t < t1; ++t) {
    in = tile_records(src, t, c);
    if (c) break;
  }
  if (t >= t1) return;
  uint64_t cur[kRadixR];
  tiles_load_round(in, j, c, cur);
  for (;;) {
    // the next round: further in this tile, else the next tile with records
    uint64_t nt = t;
    uint32_t nj = j + 64u * kRadixR, nc = c;
    const uint64_t *nin = in;
    if (nj >= c) {
      nj = 0;
      for (++nt; nt < t1; ++nt) {
        nin = tile_records(src, nt, nc);
        if (nc) break;
      }
    }
    const bool more = nt < t1;
    uint64_t nxt[kRadixR];
    // after the last round this reloads the current one (not used)
    tiles_load_round(more ? nin : in, more ? nj : j, more ? nc : c, nxt);
#pragma unroll
    for (int u = 0; u < kRadixR; ++u) {
      if (j + (uint32_t)u * 64u + lane >= c) continue;
      const uint64_t rec = cur[u];
      const uint32_t dg = (uint32_t)(rec >> kPosBits) & (ND - 1u);
      atomicOr(&grp[dg], (unsigned long long)me);
      const uint64_t peers = grp[dg];
      const uint64_t at = run[dg];
      out[at + __builtin_popcountll(peers & lt_mask)] = rec & kPosMask;
      if ((peers >> lane) == 1ull) {
        run[dg] = at + __builtin_popcountll(peers);
        grp[dg] = 0;
      }
    }
    if (!more) break;
#pragma unroll
    for (int u = 0; u < kRadixR; ++u) cur[u] = nxt[u];
    t = nt;
    j = nj;
    c = nc;
    in = nin;
  }
}

// Start of every (digit, block) of a one-pass sort from its block-major
// histogram h[b][d] (nblk blocks, nd digits).  The blocks go in chunks of
// kDigitChunk: digit_chunk_sums sums each chunk's rows (csum[c][d]);
// digit_chunk_starts scans every digit's column over the chunks (crel[c][d]:
// the counts of digit d in the chunks before c) and writes the digit totals;
// digit_block_starts scans the totals across digits (where each digit starts)
// and writes goff[b][d] = that start + crel + the counts of digit d in the
// chunk's blocks before b.  Every access walks rows, 64 lanes over
// consecutive digits.
constexpr uint32_t kDigitChunk = 32;
constexpr uint32_t kDigitWaves = 4;  // waves of digit_chunk_starts, one block per 64 digits

__global__ __launch_bounds__(256) void digit_chunk_sums(const uint32_t *__restrict__ h, uint64_t nblk, uint32_t nd,
                                                        uint32_t *__restrict__ csum) {
  const uint64_t b0 = (uint64_t)blockIdx.x * kDigitChunk, b1 = min(b0 + kDigitChunk, nblk);
  for (uint32_t d = threadIdx.x; d < nd; d += 256) {
    uint32_t t = 0;
#pragma unroll 8
    for (uint64_t b = b0; b < b1; ++b) t += h[b * nd + d];
    csum[(uint64_t)blockIdx.x * nd + d] = t;
  }
}

// Block x covers digits 64x..64x+63 (one per lane); wave w takes a
// contiguous run of chunks, sums it, then writes its chunks' exclusive
// column prefixes from the sums of the waves before it.
__global__ __launch_bounds__(64 * kDigitWaves) void digit_chunk_starts(const uint32_t *__restrict__ csum,
                                                                        uint64_t nchunk, uint32_t nd,
                                                                        uint64_t *__restrict__ crel,
                                                                        uint64_t *__restrict__ dtot) {
  __shared__ uint64_t part[kDigitWaves][64];
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t d = blockIdx.x * 64 + lane;
  const uint64_t per = (nchunk + kDigitWaves - 1) / kDigitWaves;
  const uint64_t c0 = min((uint64_t)w * per, nchunk), c1 = min(c0 + per, nchunk);
  uint64_t t = 0;
  if (d < nd)
#pragma unroll 8
    for (uint64_t c = c0; c < c1; ++c) t += csum[c * nd + d];
  part[w][lane] = t;
  __syncthreads();
  uint64_t run = 0;
  for (uint32_t i = 0; i < w; ++i) run += part[i][lane];
  if (d < nd) {
    for (uint64_t c = c0; c < c1; ++c) {
      crel[c * nd + d] = run;
      run += csum[c * nd + d];
    }
    if (w == kDigitWaves - 1) dtot[d] = run;
  }
}

// Chunk x's blocks, digits 256y..256y+255.  Every block scans the digit
// totals itself (nd is at most 2048); block (0, 0) also writes offsets (the digit is the whole pid of a
// one-pass sort): offsets[j] = start of pid j, offsets[k] = n.
__global__ __launch_bounds__(256) void digit_block_starts(const uint32_t *__restrict__ h, uint64_t nblk, uint32_t nd,
                                                          const uint64_t *__restrict__ crel,
                                                          const uint64_t *__restrict__ dtot,
                                                          uint64_t *__restrict__ goff, uint32_t k, uint64_t n,
                                                          uint64_t *__restrict__ offsets) {
  constexpr uint32_t kPer = 8;  // digits per thread of the totals' scan (256 * 8 = 2048)
  __shared__ uint64_t start[256 * kPer];
  __shared__ uint64_t wsum[4];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t v[kPer], x = 0;
#pragma unroll
  for (uint32_t i = 0; i < kPer; ++i) {
    const uint32_t d = threadIdx.x * kPer + i;
    v[i] = d < nd ? dtot[d] : 0;
    x += v[i];
  }
  const uint64_t mine = x;
  for (int sh = 1; sh < 64; sh <<= 1) {
    const uint64_t y = __shfl_up(x, sh, 64);
    if (lane >= (uint32_t)sh) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint64_t before = x - mine;
  for (uint32_t i = 0; i < wave; ++i) before += wsum[i];
#pragma unroll
  for (uint32_t i = 0; i < kPer; ++i) {
    start[threadIdx.x * kPer + i] = before;
    before += v[i];
  }
  __syncthreads();
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (uint32_t j = threadIdx.x; j <= k; j += 256) offsets[j] = j < k ? start[j] : n;
  const uint64_t b0 = (uint64_t)blockIdx.x * kDigitChunk, b1 = min(b0 + kDigitChunk, nblk);
  const uint32_t d = blockIdx.y * 256 + threadIdx.x;
  if (d >= nd) return;
  uint64_t run = start[d] + crel[(uint64_t)blockIdx.x * nd + d];
  uint32_t c[kDigitChunk];
#pragma unroll
  for (uint32_t i = 0; i < kDigitChunk; ++i) c[i] = b0 + i < b1 ? h[(b0 + i) * nd + d] : 0;
#pragma unroll
  for (uint32_t i = 0; i < kDigitChunk; ++i) {
    if (b0 + i < b1) goff[(b0 + i) * nd + d] = run;
    run += c[i];
  }
}

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
  return 2 * tile + kCandCap * 2 + 64 * 4 + img_cap;  // two tile slots
}

// exclusive scan of n u32 counts into u64 offsets; tmp holds scan_tmp_words(n)
// u64; *total_dev (optional) receives the sum.
uint64_t scan_tmp_words(uint64_t n) { return (n + kScanBlock - 1) / kScanBlock + 2; }

hipError_t launch_exclusive_scan(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *tmp, uint64_t *total_dev,
                                 hipStream_t s) {
  const uint64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb > 0) hipLaunchKernelGGL(scan_block_sums, dim3((uint32_t)nb), dim3(kScanWG), 0, s, in, n, tmp);
  if (nb > 0 && nb <= (uint64_t)kScanWG) {
    hipLaunchKernelGGL((scan_local<true>), dim3((uint32_t)nb), dim3(kScanWG), 0, s, in, n, tmp, nb, out, total_dev);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(scan_sums_single, dim3(1), dim3(kScanWG), 0, s, tmp, nb, total_dev);
  if (nb > 0)
    hipLaunchKernelGGL((scan_local<false>), dim3((uint32_t)nb), dim3(kScanWG), 0, s, in, n, tmp, nb, out, nullptr);
  return hipGetLastError();
}

hipError_t launch_exclusive_scan_summed(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *bsum, hipStream_t s) {
  static_assert(kScanBlock == (1 << kTileSumLog2), "the count pass sums the scan's blocks");
  const uint64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb == 0) return hipSuccess;
  if (nb <= (uint64_t)kScanWG) {
    hipLaunchKernelGGL((scan_local<true>), dim3((uint32_t)nb), dim3(kScanWG), 0, s, in, n, bsum, nb, out, nullptr);
  } else {
    hipLaunchKernelGGL(scan_sums_single, dim3(1), dim3(kScanWG), 0, s, bsum, nb, nullptr);
    hipLaunchKernelGGL((scan_local<false>), dim3((uint32_t)nb), dim3(kScanWG), 0, s, in, n, bsum, nb, out, nullptr);
  }
  return hipGetLastError();
}

hipError_t launch_compact(const uint32_t *counts, const uint64_t *offs, uint64_t ntiles, const uint64_t *slabs,
                          uint32_t slab_cap, uint64_t *out, bool sparse, uint64_t *offsets1, uint64_t total,
                          hipStream_t s) {
  if (ntiles == 0) return hipSuccess;
  if (sparse)
    hipLaunchKernelGGL(compact_sparse, dim3((uint32_t)((ntiles + 255) / 256)), dim3(256), 0, s, counts, offs, ntiles,
                       slabs, slab_cap, out, offsets1, total);
  else
    hipLaunchKernelGGL(compact_slabs, dim3((uint32_t)((ntiles + 3) / 4)), dim3(256), 0, s, counts, offs, ntiles,
                       slabs, slab_cap, out, offsets1, total);
  return hipGetLastError();
}

uint64_t radix_blocks(uint64_t n) { return (n + kRadixBlock - 1) / kRadixBlock; }

// Starts of every (digit, block) of a one-pass sort into goff (block-major,
// like h) and of every digit into offsets (k + 1 entries); cs: work of
// digit_cs_bytes(nblk * nd, nd) bytes.
static hipError_t digit_offsets(const uint32_t *h, uint64_t nblk, uint32_t nd, uint64_t *goff, uint8_t *cs,
                                uint32_t k, uint64_t n, uint64_t *offsets, hipStream_t s) {
  if (nd > 2048 || k > nd) return hipErrorInvalidValue;
  const uint64_t nchunk = (nblk + kDigitChunk - 1) / kDigitChunk;
  uint32_t *csum = (uint32_t *)cs;
  uint64_t *crel = (uint64_t *)(cs + ((nchunk * nd * 4 + 255) & ~255ull));
  uint64_t *dtot = crel + nchunk * nd;
  hipLaunchKernelGGL(digit_chunk_sums, dim3((uint32_t)nchunk), dim3(256), 0, s, h, nblk, nd, csum);
  hipLaunchKernelGGL(digit_chunk_starts, dim3((nd + 63) / 64), dim3(64 * kDigitWaves), 0, s, csum, nchunk, nd, crel,
                     dtot);
  hipLaunchKernelGGL(digit_block_starts, dim3((uint32_t)nchunk, (nd + 255) / 256), dim3(256), 0, s, h, nblk, nd, crel,
                     dtot, goff, k, n, offsets);
  return hipGetLastError();
}

uint64_t digit_cs_bytes(uint64_t nh, uint32_t nd) {
  const uint64_t cells = nh / kDigitChunk + nd;  // at least nchunk * nd for any nblk * nd <= nh
  return ((cells * 4 + 255) & ~255ull) + cells * 8 + nd * 8;
}

template <int DB>
static hipError_t radix_one_pass(const uint64_t *src, uint64_t n, uint32_t k, uint32_t *ghist, uint64_t *goff,
                                 uint8_t *cs, uint64_t *offsets, uint64_t *positions, hipStream_t s) {
  constexpr int BLK = DB == 8 ? kRadixBlock : kRadixBlock11;
  const uint64_t nblk = (n + BLK - 1) / BLK;
  hipLaunchKernelGGL((radix_hist<DB, BLK, true>), dim3((uint32_t)nblk), dim3(64), 0, s, src, n, kPosBits, ghist,
                     nblk);
  hipError_t e = digit_offsets(ghist, nblk, 1u << DB, goff, cs, k, n, offsets, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((radix_scatter<DB, BLK, true, true>), dim3((uint32_t)nblk), dim3(64), 0, s, src, n, kPosBits,
                     goff, nblk, positions);
  return hipGetLastError();
}

// Stable sort of n records by pid (bits 40.. of each record, pids below k),
// written out as per-pid offsets (k+1) and positions (n).  Up to 2,048 pids:
// one pass whose digit is the whole pid, scattering positions straight to
// their final place, with the offsets read from the scanned histogram.
// Beyond: 8-bit passes ping-ponging between a and b, then a binary search
// for the offsets and a strip of the records.  ghist / goff / tmp are sized
// for 256 * radix_blocks(n) entries, which also covers the one-pass digits
// (at most 2048 per 8192-record block).
hipError_t launch_radix(uint64_t *a, uint64_t *b, uint64_t n, uint32_t k, uint32_t *ghist, uint64_t *goff,
                        uint64_t *tmp, uint8_t *cs, uint64_t *offsets, uint64_t *positions, hipStream_t s) {
  uint32_t pid_bits = 0;
  while (pid_bits < 32 && (1ull << pid_bits) < k) ++pid_bits;
  if (n == 0) return hipSuccess;
  if (pid_bits <= 8) return radix_one_pass<8>(a, n, k, ghist, goff, cs, offsets, positions, s);
  if (pid_bits == 9) return radix_one_pass<9>(a, n, k, ghist, goff, cs, offsets, positions, s);
  if (pid_bits == 10) return radix_one_pass<10>(a, n, k, ghist, goff, cs, offsets, positions, s);
  if (pid_bits == 11) return radix_one_pass<11>(a, n, k, ghist, goff, cs, offsets, positions, s);
  uint64_t *src = a, *dst = b;
  const uint64_t nblk = radix_blocks(n);
  const uint32_t npass = (pid_bits + 7) / 8;
  for (uint32_t ps = 0; ps < npass; ++ps) {
    const uint32_t shift = kPosBits + 8 * ps;
    hipLaunchKernelGGL((radix_hist<8, kRadixBlock, false>), dim3((uint32_t)nblk), dim3(64), 0, s, src, n, shift, ghist,
                       nblk);
    hipError_t e = launch_exclusive_scan(ghist, 256 * nblk, goff, tmp, nullptr, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((radix_scatter<8, kRadixBlock, false, false>), dim3((uint32_t)nblk), dim3(64), 0, s, src, n, shift,
                       goff, nblk, dst);
    uint64_t *t = src;
    src = dst;
    dst = t;
  }
  hipError_t e = launch_pid_offsets(src, n, k, offsets, s);
  if (e != hipSuccess) return e;
  return launch_strip(src, n, positions, s);
}

template <int DB>
static hipError_t radix_tiles_pass(const TileSrc *parts, uint32_t nparts, uint64_t nblk, uint64_t n, uint32_t k,
                                   uint32_t *ghist, uint64_t *goff, uint8_t *cs, uint64_t *offsets,
                                   uint64_t *positions, hipStream_t s) {
  for (uint32_t i = 0; i < nparts; ++i) {
    const uint64_t nb = (parts[i].ntiles + parts[i].G - 1) / parts[i].G;
    if (nb) hipLaunchKernelGGL((radix_hist_tiles<DB>), dim3((uint32_t)nb), dim3(256), 0, s, parts[i], ghist, nblk);
  }
  hipError_t e = digit_offsets(ghist, nblk, 1u << DB, goff, cs, k, n, offsets, s);
  if (e != hipSuccess) return e;
  for (uint32_t i = 0; i < nparts; ++i) {
    const uint64_t nb = (parts[i].ntiles + parts[i].G - 1) / parts[i].G;
    if (nb)
      hipLaunchKernelGGL((radix_scatter_tiles<DB>), dim3((uint32_t)nb), dim3(64), 0, s, parts[i], goff, nblk,
                         positions);
  }
  return hipGetLastError();
}

// The one-pass sort (up to 2,048 pids) over records read from the staging
// slabs (see TileSrc); parts[i].G and blk0 set by the caller, nblk the total
// block count (the histograms hold 2^pid_bits * nblk entries).
hipError_t launch_radix_tiles(const TileSrc *parts, uint32_t nparts, uint64_t nblk, uint64_t n, uint32_t k,
                              uint32_t *ghist, uint64_t *goff, uint8_t *cs, uint64_t *offsets, uint64_t *positions,
                              hipStream_t s) {
  uint32_t pid_bits = 0;
  while (pid_bits < 32 && (1ull << pid_bits) < k) ++pid_bits;
  if (n == 0) return hipSuccess;
  if (pid_bits <= 8) return radix_tiles_pass<8>(parts, nparts, nblk, n, k, ghist, goff, cs, offsets, positions, s);
  if (pid_bits == 9) return radix_tiles_pass<9>(parts, nparts, nblk, n, k, ghist, goff, cs, offsets, positions, s);
  if (pid_bits == 10) return radix_tiles_pass<10>(parts, nparts, nblk, n, k, ghist, goff, cs, offsets, positions, s);
  if (pid_bits == 11) return radix_tiles_pass<11>(parts, nparts, nblk, n, k, ghist, goff, cs, offsets, positions, s);
  return hipErrorInvalidValue;
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


hipError_t launch_window_hashes(const uint8_t *text, uint64_t n, uint32_t m, const uint64_t *xs, uint64_t cnt,
                                uint64_t *out, hipStream_t s) {
  if (cnt == 0) return hipSuccess;
  hipLaunchKernelGGL(window_hashes_kernel, dim3((uint32_t)((cnt + 255) / 256)), dim3(256), 0, s, text, n, m, xs, cnt,
                     out);
  return hipGetLastError();
}

// --------------------------------------------------------- scan dispatch
#define RK_SCAN_DISPATCH(fam, cfg, CALL)                       \
  switch (fam * 16 + cfg) {                                    \
    case kFamScreen1 * 16 + 0: return ScanGeom<kFamScreen1, 0>::CALL; \
    case kFamScreen1 * 16 + 1: return ScanGeom<kFamScreen1, 1>::CALL; \
    case kFamScreen1 * 16 + 2: return ScanGeom<kFamScreen1, 2>::CALL; \
    case kFamScreen1 * 16 + 3: return ScanGeom<kFamScreen1, 3>::CALL; \
    case kFamScreen * 16 + 0: return ScanGeom<kFamScreen, 0>::CALL;   \
    case kFamScreen * 16 + 1: return ScanGeom<kFamScreen, 1>::CALL;   \
    case kFamScreen * 16 + 2: return ScanGeom<kFamScreen, 2>::CALL;   \
    case kFamScreen * 16 + 3: return ScanGeom<kFamScreen, 3>::CALL;   \
    case kFamExact * 16 + 0: return ScanGeom<kFamExact, 0>::CALL;     \
    case kFamExact * 16 + 1: return ScanGeom<kFamExact, 1>::CALL;     \
    case kFamExact * 16 + 2: return ScanGeom<kFamExact, 2>::CALL;     \
    case kFamExact * 16 + 3: return ScanGeom<kFamExact, 3>::CALL;     \
    default: return hipErrorInvalidValue;                      \
  }

hipError_t scan_occupancy(int cfg, int fam, uint32_t lds_bytes, int *blocks) {
  RK_SCAN_DISPATCH(fam, cfg, occupancy(lds_bytes, blocks))
}

hipError_t launch_scan(int cfg, int fam, const ScanParams &p, uint32_t grid, uint32_t lds_bytes, hipStream_t s) {
  RK_SCAN_DISPATCH(fam, cfg, launch(p, grid, lds_bytes, s))
}

// Launches (p != nullptr) or sizes (occupancy into *blocks) the single-bucket
// scan of geometry cfg and family fam.
hipError_t list_scan(int cfg, int fam, const ListParams *p, uint32_t grid, hipStream_t s, int *blocks) {
  RK_SCAN_DISPATCH(fam, cfg, list(p, grid, s, blocks))
}

static hipError_t prepare_scan_kernel(int fam, int cfg) { RK_SCAN_DISPATCH(fam, cfg, prepare()) }
static hipError_t prepare_list_kernel(int fam, int cfg) { RK_SCAN_DISPATCH(fam, cfg, list_prepare()) }

// Raises the dynamic LDS limit of every scan kernel once, outside any stream
// capture (a graph capture must not run first-time setup calls).
void prepare_scan_kernels() {
  for (int fam : {kFamScreen1, kFamScreen, kFamExact})
    for (int cfg = 0; cfg < kNumTileCfg; ++cfg) {
      (void)prepare_scan_kernel(fam, cfg);
      (void)prepare_list_kernel(fam, cfg);
    }
}

// ----------------------------------------------------- stream-read roofline
// Reads every 16-byte block of data[0..n) once (the scan's load width, fully
// coalesced, grid-stride) and folds it into one word per workgroup so that
// nothing is optimised away: the read-bandwidth ceiling the scan is held to.
// Each wave streams 1 KiB chunks (gw, gw + TW, ...; TW waves in the grid)
// into a private LDS ring of two sets of 8 slots with non-temporal LDS-DMA
// loads, the way the scans load their tiles: a batch of 8 is issued, then the
// previous batch is waited for and XOR-folded from LDS (every byte is read).
// Tail bytes (n % 1024) are folded by the first workgroup's first wave.
__device__ __forceinline__ uint32_t sr_lds(const void *p) {
  return (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const uint8_t *)p;
}

__device__ __forceinline__ void sr_dma(const void *g, uint32_t m0) {
  __asm__ volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off nt" ::"v"(g), "{m0}"(m0) : "memory");
}

__global__ __launch_bounds__(256) void stream_read_kernel(const uint8_t *data, uint64_t n, uint32_t *out) {
  __shared__ __attribute__((aligned(16))) uint8_t ring[4][2][8][1024];
  const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t nchunks = n / 1024, gw = (uint64_t)blockIdx.x * 4 + w, tw = (uint64_t)gridDim.x * 4;
  uint32_t acc = 0, par = 0, prev = 0;
  for (uint64_t c0 = gw; c0 < nchunks; c0 += 8 * tw) {
    // the previous batch's reads of the set about to be refilled are done
    __asm__ volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    uint32_t cnt = 0;
#pragma unroll
    for (uint32_t j = 0; j < 8; ++j) {
      const uint64_t c = c0 + j * tw;
      if (c < nchunks) {
        sr_dma(data + c * 1024 + 16 * lane, __builtin_amdgcn_readfirstlane(sr_lds(&ring[w][par][j][0])));
        ++cnt;
      }
    }
    if (cnt == 8)
      __builtin_amdgcn_s_waitcnt(0x0F78);  // vmcnt(8): the previous batch has landed
    else
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    __asm__ volatile("" ::: "memory");
    for (uint32_t j = 0; j < prev; ++j) {
      const uint4 v = *(const uint4 *)&ring[w][par ^ 1][j][16 * lane];
      acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    prev = cnt;
    par ^= 1;
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);
  __asm__ volatile("" ::: "memory");
  for (uint32_t j = 0; j < prev; ++j) {
    const uint4 v = *(const uint4 *)&ring[w][par ^ 1][j][16 * lane];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  if (blockIdx.x == 0 && w == 0 && nchunks * 1024 + 16 * lane < n) {
    const uint4 v = *(const uint4 *)(data + nchunks * 1024 + 16 * lane);
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  for (int d = 32; d >= 1; d >>= 1) acc ^= __shfl_xor(acc, d, 64);
  __shared__ uint32_t red[4];
  if (lane == 0) red[w] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = red[0] ^ red[1] ^ red[2] ^ red[3];
}

hipError_t launch_stream_read(const void *data, uint64_t n, uint32_t *out, uint32_t grid, hipStream_t s) {
  hipLaunchKernelGGL(stream_read_kernel, dim3(grid), dim3(256), 0, s, (const uint8_t *)data, n, out);
  return hipGetLastError();
}

}  // namespace rk
