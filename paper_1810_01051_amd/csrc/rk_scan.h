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
//            shift out and no out-term is needed) and compared with the set.
// A candidate window (its hash passed the set test) is hashed again from
// scratch (exact: Horner, canonical value; screen: shift-and-add), looked up
// in the open-addressing table of its bucket and confirmed byte by byte
// against every pattern chained under that hash.
//
// Hits are compacted with a block-wide prefix sum in ascending window order per
// bucket into a per-tile staging slab; later kernels scan the tile counts,
// compact the slabs and sort stably by pattern id.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rk_dev.h"
#include "rk_internal.h"
#include "rk_runtime.h"

namespace rk {

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

typedef __attribute__((address_space(3))) const uint32_t lds_word;

// ---------------------------------------------------- LDS reads out of sight
// The tile pipeline issues the next tiles' loads-to-LDS before testing the
// current tile.  The compiler cannot tell that the current tile's LDS words
// are not the ones those loads write, so before any LDS read it can see it
// waits for every outstanding load -- the next tiles' included, which would
// end the overlap.  The tile words are therefore read by inline asm (pairs of
// dwords, then one wait for all of them inside the same statement, so that no
// word is used before it has arrived; the outputs are early-clobber, as the
// address is still read after the first word is written); the explicit
// barriers of the pipeline order these reads after the tile has landed.
typedef uint32_t rk_u32x2 __attribute__((ext_vector_type(2)));

#define RK_DSP1 "ds_read2_b32 %0, %[a] offset0:0 offset1:1\n"
#define RK_DSP2 RK_DSP1 "ds_read2_b32 %1, %[a] offset0:2 offset1:3\n"
#define RK_DSP3 RK_DSP2 "ds_read2_b32 %2, %[a] offset0:4 offset1:5\n"
#define RK_DSP4 RK_DSP3 "ds_read2_b32 %3, %[a] offset0:6 offset1:7\n"
#define RK_DSP5 RK_DSP4 "ds_read2_b32 %4, %[a] offset0:8 offset1:9\n"
#define RK_DSP6 RK_DSP5 "ds_read2_b32 %5, %[a] offset0:10 offset1:11\n"
#define RK_DSP7 RK_DSP6 "ds_read2_b32 %6, %[a] offset0:12 offset1:13\n"
#define RK_DSP8 RK_DSP7 "ds_read2_b32 %7, %[a] offset0:14 offset1:15\n"
#define RK_DSP9 RK_DSP8 "ds_read2_b32 %8, %[a] offset0:16 offset1:17\n"
#define RK_DSP10 RK_DSP9 "ds_read2_b32 %9, %[a] offset0:18 offset1:19\n"
#define RK_DSP11 RK_DSP10 "ds_read2_b32 %10, %[a] offset0:20 offset1:21\n"
#define RK_DSP12 RK_DSP11 "ds_read2_b32 %11, %[a] offset0:22 offset1:23\n"
#define RK_DSP13 RK_DSP12 "ds_read2_b32 %12, %[a] offset0:24 offset1:25\n"
#define RK_DSP14 RK_DSP13 "ds_read2_b32 %13, %[a] offset0:26 offset1:27\n"
#define RK_DSP15 RK_DSP14 "ds_read2_b32 %14, %[a] offset0:28 offset1:29\n"
#define RK_DSP16 RK_DSP15 "ds_read2_b32 %15, %[a] offset0:30 offset1:31\n"
#define RK_DSP17 RK_DSP16 "ds_read2_b32 %16, %[a] offset0:32 offset1:33\n"
#define RK_DSP18 RK_DSP17 "ds_read2_b32 %17, %[a] offset0:34 offset1:35\n"
#define RK_DSP19 RK_DSP18 "ds_read2_b32 %18, %[a] offset0:36 offset1:37\n"
#define RK_DSP20 RK_DSP19 "ds_read2_b32 %19, %[a] offset0:38 offset1:39\n"
#define RK_DSP21 RK_DSP20 "ds_read2_b32 %20, %[a] offset0:40 offset1:41\n"
#define RK_DSP22 RK_DSP21 "ds_read2_b32 %21, %[a] offset0:42 offset1:43\n"
#define RK_DSP23 RK_DSP22 "ds_read2_b32 %22, %[a] offset0:44 offset1:45\n"
#define RK_DSP24 RK_DSP23 "ds_read2_b32 %23, %[a] offset0:46 offset1:47\n"
#define RK_DSO1(v) "=&v"(v[0])
#define RK_DSO2(v) RK_DSO1(v), "=&v"(v[1])
#define RK_DSO3(v) RK_DSO2(v), "=&v"(v[2])
#define RK_DSO4(v) RK_DSO3(v), "=&v"(v[3])
#define RK_DSO5(v) RK_DSO4(v), "=&v"(v[4])
#define RK_DSO6(v) RK_DSO5(v), "=&v"(v[5])
#define RK_DSO7(v) RK_DSO6(v), "=&v"(v[6])
#define RK_DSO8(v) RK_DSO7(v), "=&v"(v[7])
#define RK_DSO9(v) RK_DSO8(v), "=&v"(v[8])
#define RK_DSO10(v) RK_DSO9(v), "=&v"(v[9])
#define RK_DSO11(v) RK_DSO10(v), "=&v"(v[10])
#define RK_DSO12(v) RK_DSO11(v), "=&v"(v[11])
#define RK_DSO13(v) RK_DSO12(v), "=&v"(v[12])
#define RK_DSO14(v) RK_DSO13(v), "=&v"(v[13])
#define RK_DSO15(v) RK_DSO14(v), "=&v"(v[14])
#define RK_DSO16(v) RK_DSO15(v), "=&v"(v[15])
#define RK_DSO17(v) RK_DSO16(v), "=&v"(v[16])
#define RK_DSO18(v) RK_DSO17(v), "=&v"(v[17])
#define RK_DSO19(v) RK_DSO18(v), "=&v"(v[18])
#define RK_DSO20(v) RK_DSO19(v), "=&v"(v[19])
#define RK_DSO21(v) RK_DSO20(v), "=&v"(v[20])
#define RK_DSO22(v) RK_DSO21(v), "=&v"(v[21])
#define RK_DSO23(v) RK_DSO22(v), "=&v"(v[22])
#define RK_DSO24(v) RK_DSO23(v), "=&v"(v[23])

// reads NW consecutive dwords at LDS byte address a (4-byte aligned) into w
template <int NW>
__device__ __forceinline__ void lds_read_words(uint32_t *w, uint32_t a) {
  constexpr int P = NW / 2;
  static_assert(NW >= 2 && P <= 24, "word count within the generated forms");
  rk_u32x2 v[P];
  uint32_t last = 0;
  (void)last;
  if constexpr (P == 1) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP1 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO1(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP1 "s_waitcnt lgkmcnt(0)" : RK_DSO1(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 2) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP2 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO2(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP2 "s_waitcnt lgkmcnt(0)" : RK_DSO2(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 3) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP3 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO3(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP3 "s_waitcnt lgkmcnt(0)" : RK_DSO3(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 4) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP4 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO4(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP4 "s_waitcnt lgkmcnt(0)" : RK_DSO4(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 5) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP5 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO5(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP5 "s_waitcnt lgkmcnt(0)" : RK_DSO5(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 6) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP6 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO6(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP6 "s_waitcnt lgkmcnt(0)" : RK_DSO6(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 7) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP7 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO7(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP7 "s_waitcnt lgkmcnt(0)" : RK_DSO7(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 8) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP8 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO8(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP8 "s_waitcnt lgkmcnt(0)" : RK_DSO8(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 9) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP9 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO9(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP9 "s_waitcnt lgkmcnt(0)" : RK_DSO9(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 10) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP10 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO10(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP10 "s_waitcnt lgkmcnt(0)" : RK_DSO10(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 11) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP11 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO11(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP11 "s_waitcnt lgkmcnt(0)" : RK_DSO11(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 12) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP12 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO12(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP12 "s_waitcnt lgkmcnt(0)" : RK_DSO12(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 13) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP13 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO13(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP13 "s_waitcnt lgkmcnt(0)" : RK_DSO13(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 14) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP14 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO14(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP14 "s_waitcnt lgkmcnt(0)" : RK_DSO14(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 15) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP15 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO15(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP15 "s_waitcnt lgkmcnt(0)" : RK_DSO15(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 16) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP16 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO16(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP16 "s_waitcnt lgkmcnt(0)" : RK_DSO16(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 17) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP17 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO17(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP17 "s_waitcnt lgkmcnt(0)" : RK_DSO17(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 18) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP18 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO18(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP18 "s_waitcnt lgkmcnt(0)" : RK_DSO18(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 19) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP19 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO19(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP19 "s_waitcnt lgkmcnt(0)" : RK_DSO19(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 20) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP20 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO20(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP20 "s_waitcnt lgkmcnt(0)" : RK_DSO20(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 21) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP21 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO21(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP21 "s_waitcnt lgkmcnt(0)" : RK_DSO21(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 22) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP22 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO22(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP22 "s_waitcnt lgkmcnt(0)" : RK_DSO22(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 23) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP23 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO23(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP23 "s_waitcnt lgkmcnt(0)" : RK_DSO23(v) : [a] "v"(a) : "memory");
  } else if constexpr (P == 24) {
    if constexpr (NW & 1)
      __asm__ volatile(RK_DSP24 "ds_read_b32 %[l], %[a] offset:%[o]\n\ts_waitcnt lgkmcnt(0)"
                       : RK_DSO24(v), [l] "=&v"(last) : [a] "v"(a), [o] "n"(8 * P) : "memory");
    else
      __asm__ volatile(RK_DSP24 "s_waitcnt lgkmcnt(0)" : RK_DSO24(v) : [a] "v"(a) : "memory");
  }
#pragma unroll
  for (int j = 0; j < P; ++j) {
    w[2 * j] = v[j].x;
    w[2 * j + 1] = v[j].y;
  }
  if constexpr (NW & 1) w[NW - 1] = last;
}

__device__ __forceinline__ uint32_t lds_addr(const void *p) { return (uint32_t)(uintptr_t)(lds_word *)p; }

// The thread's bytes, loaded from the LDS tile by each pass itself (so that
// the loads, and the byte extractions that follow them, are not shared between
// the test variants of a bucket and hoisted above the variant switch, which
// would keep every extracted byte of every variant live at once; no register
// copy of the words stays live across buckets either).
template <int NW>
__device__ __forceinline__ void load_words(uint32_t *w, const uint32_t *tw) {
  lds_read_words<NW>(w, lds_addr(tw));
}

// The thread's words of a tile already in registers (the 64 bytes before its
// first window end and its C bytes; for exact passes also the out-stream
// dwords), or none (nullptr): then each pass reads them from the LDS tile.
template <int C>
struct PreWords {
  uint32_t w[16 + C / 4];
  uint32_t d[C / 4 + 1];
};

// Shift-add hash state after the 64 bytes held in w[0..16), i.e. before the
// thread's first window end: h = sum_j b[63-j] << (S*j) mod 2^32 (bytes older
// than 32/S positions have shifted out).  For S = 2 four bytes at a time with
// one dot product each: the weights 4^3..4^0 of a word's bytes fit in bytes.
template <int S>
__device__ __forceinline__ uint32_t screen_init(const uint32_t *w) {
  if constexpr (S == 2) {
    uint32_t h = 0;
#pragma unroll
    for (int q = 12; q < 16; ++q) h = __builtin_amdgcn_udot4(w[q], 0x01041040u, h << 8, false);
    return h;
  } else {
    constexpr int WU = 32 / S - 1;  // bytes before the first window end that are still in the hash
    uint32_t h = 0;
#pragma unroll
    for (int j = 64 - WU; j < 64; ++j) h = (h << S) + byte_at(w, j);
    return h;
  }
}

// OR of the wave ballots, kept as a sequential chain of scalar ORs (a
// reassociated OR tree would keep one SGPR pair per window alive).
__device__ __forceinline__ void any_or(uint64_t &any, uint64_t b) {
  any |= b;
  __asm__ volatile("" : "+s"(any));
}

template <int C, int S, int NT, bool ANY>
__device__ __forceinline__ void pass_list_screen_w(const uint32_t *w, uint32_t msk, const uint32_t *tg, uint64_t &any,
                                                   Bits<C> &bits) {
  uint32_t h = screen_init<S>(w), acc = 0;
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

// The words come from registers (pre) or from the LDS tile; each branch
// passes its own register array, so that no pointer selects between them.
template <int C, int S, int NT, bool ANY, bool PRE>
__device__ __forceinline__ void pass_list_screen(const uint32_t *tw, uint32_t msk, const uint32_t *tg, uint64_t &any,
                                                 Bits<C> &bits, const PreWords<C> *pre) {
  if constexpr (PRE) {
    pass_list_screen_w<C, S, NT, ANY>(pre->w, msk, tg, any, bits);
  } else {
    uint32_t w[16 + C / 4];
    load_words<16 + C / 4>(w, tw);
    pass_list_screen_w<C, S, NT, ANY>(w, msk, tg, any, bits);
  }
}

// Set test against a cuckoo table in LDS: the key is in one of its two slots.
__device__ __forceinline__ bool in_cuckoo(const uint32_t *tab, uint32_t sh, uint32_t h) {
  return (tab[ck_slot1(h, sh)] == h) | (tab[ck_slot2(h, sh)] == h);
}

// Windows per block of the table tests: the LDS probes of a block's windows
// are all issued before the first of them is compared, so that their
// latencies overlap (C is a multiple of 4 in every geometry).
constexpr int kProbeBlock = 4;

template <int C, int S, bool ANY>
__device__ __forceinline__ void pass_table_screen_w(const uint32_t *w, uint32_t msk, const uint32_t *tab, uint32_t sh,
                                                    uint64_t &any, Bits<C> &bits) {
  static_assert(C % kProbeBlock == 0, "whole probe blocks");
  uint32_t h = screen_init<S>(w), acc = 0;
#pragma unroll
  for (int i0 = 0; i0 < C; i0 += kProbeBlock) {
    uint32_t v[kProbeBlock], t1[kProbeBlock], t2[kProbeBlock];
#pragma unroll
    for (int j = 0; j < kProbeBlock; ++j) {
      h = (h << S) + byte_at(w, 64 + i0 + j);
      v[j] = (S == 8) ? (h & msk) : h;
    }
#pragma unroll
    for (int j = 0; j < kProbeBlock; ++j) {
      t1[j] = tab[ck_slot1(v[j], sh)];
      t2[j] = tab[ck_slot2(v[j], sh)];
    }
    if (ANY) {
      uint64_t b = 0;
#pragma unroll
      for (int j = 0; j < kProbeBlock; ++j) b |= ballot(t1[j] == v[j]) | ballot(t2[j] == v[j]);
      any_or(any, b);
    } else {
#pragma unroll
      for (int j = 0; j < kProbeBlock; ++j) put_bit<C>(bits, acc, i0 + j, (t1[j] == v[j]) | (t2[j] == v[j]));
    }
  }
}

template <int C, int S, bool ANY, bool PRE>
__device__ __forceinline__ void pass_table_screen(const uint32_t *tw, uint32_t msk, const uint32_t *tab, uint32_t sh,
                                                  uint64_t &any, Bits<C> &bits, const PreWords<C> *pre) {
  if constexpr (PRE) {
    pass_table_screen_w<C, S, ANY>(pre->w, msk, tab, sh, any, bits);
  } else {
    uint32_t w[16 + C / 4];
    load_words<16 + C / 4>(w, tw);
    pass_table_screen_w<C, S, ANY>(w, msk, tab, sh, any, bits);
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
    if (lead >= 4) continue;                // wholly before the window: s stays 0 (m is uniform)
    const uint32_t keep = lead <= 0 ? 0xFFFFFFFFu : (0xFFFFFFFFu >> (8 * lead));
    s = mul2p32_lazy(s) + (__builtin_bswap32(w[q]) & keep);
  }
  return s;
}

// One exact rolling step: H(e) = 256 H(e-1) + in - out * 2^r  (r = 8m mod 61),
// with the 32-bit halves spelled out and the outgoing term specialised on
// where out * 2^r lands in the 61-bit word (r = 8m mod 61 is fixed per group):
// OUTK 0: bits r..r+7 in the low word (r <= 24), 1: in the high word
// (32 <= r <= 53), 2: anywhere (general rotation).
//   256 s mod q = ((s << 8) & q) + (s >> 53): the low byte of s << 8 is free
//   for the entering byte (byte k of the word inw, merged by one byte
//   permute); q - v = q ^ v for v <= q.
// The sum (256 s + in) + (q - out * 2^r) + (s >> 53) is two add-with-carry
// pairs (OUTK 0, 1).  s < 2^63 in, s < 2^62 + 2^11 out.
template <int OUTK>
__device__ __forceinline__ uint64_t exact_step_k(uint64_t s, uint32_t inw, uint32_t k, uint32_t out, uint32_t r) {
  const uint32_t lo = (uint32_t)s, hi = (uint32_t)(s >> 32);
  const uint32_t alo = __builtin_amdgcn_perm(lo, inw, 0x06050400u | k);  // (lo << 8) | byte k of inw
  const uint32_t ahi = __builtin_amdgcn_alignbit(hi, lo, 24) & 0x1FFFFFFFu;
  const uint32_t f = hi >> 21;
  if constexpr (OUTK == 2) {
    const uint64_t neg = kQ - rot61(out, r);
    return ((((uint64_t)ahi << 32) | alo) + neg) + f;
  } else {
    uint32_t x, h;
    if constexpr (OUTK == 0) {
      // (the high word of q comes in a VGPR: with the carry in VCC a literal
      // would be a second constant-bus read)
      __asm__("v_add_co_u32 %0, vcc, %2, %3\n\t"
              "v_addc_co_u32 %1, vcc, %6, %4, vcc\n\t"
              "v_add_co_u32 %0, vcc, %0, %5\n\t"
              "v_addc_co_u32 %1, vcc, 0, %1, vcc"
              : "=&v"(x), "=&v"(h)
              : "v"(alo), "v"(~(out << r)), "v"(ahi), "v"(f), "v"(0x1FFFFFFFu)
              : "vcc");
    } else {
      __asm__("v_add_co_u32 %0, vcc, -1, %2\n\t"
              "v_addc_co_u32 %1, vcc, %3, %4, vcc\n\t"
              "v_add_co_u32 %0, vcc, %0, %5\n\t"
              "v_addc_co_u32 %1, vcc, 0, %1, vcc"
              : "=&v"(x), "=&v"(h)
              : "v"(alo), "v"(0x1FFFFFFFu ^ (out << (r - 32))), "v"(ahi), "v"(f)
              : "vcc");
    }
    return ((uint64_t)h << 32) | x;
  }
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

// The exact rolling hash over the thread's C windows, the one loop every
// exact pass and the hash dump run: the state of the window ending before the
// thread's first one (exact_init), then one exact_step_k per window with the
// entering byte from w and the leaving byte from the out-stream dwords d;
// visit(i, s) sees the lazy state s of window i (congruent to its hash,
// s < 2^62 + 2^11).
template <int C, int OUTK, typename Visit>
__device__ __forceinline__ void roll_exact(const uint32_t *w, const uint32_t *d, OutStream os, uint32_t m, uint32_t r,
                                           Visit &&visit) {
  uint64_t s = exact_init(w, m);
  uint32_t dlo = d[0], ow = 0;
#pragma unroll
  for (int i = 0; i < C; ++i) {
    if ((i & 3) == 0) {
      const uint32_t dhi = d[(i >> 2) + 1];
      ow = __builtin_amdgcn_alignbyte(dhi, dlo, os.sh);
      dlo = dhi;
    }
    s = exact_step_k<OUTK>(s, w[(64 + i) >> 2], (uint32_t)(i & 3), (ow >> (8 * (i & 3))) & 0xFFu, r);
    visit(i, s);
  }
}

template <int C, bool ANY, bool TABLE, int NT, int OUTK>
__device__ __forceinline__ void pass_exact_w(const uint32_t *w, const uint32_t *d, OutStream os, uint32_t m, uint32_t r,
                                             const uint32_t *tg, const uint32_t *fp, uint32_t sh, uint64_t &any,
                                             Bits<C> &bits) {
  uint32_t acc = 0;
  roll_exact<C, OUTK>(w, d, os, m, r, [&](int i, uint64_t s) __attribute__((always_inline)) {
    if (TABLE) {
      const bool c = in_cuckoo(fp, sh, (uint32_t)canon(s));
      if (ANY) any_or(any, ballot(c));
      else put_bit<C>(bits, acc, i, c);
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
  });
}

template <int C, bool ANY, bool TABLE, int NT, int OUTK, bool PRE>
__device__ __forceinline__ void pass_exact(const uint32_t *tw, OutStream os, uint32_t m, uint32_t r, const uint32_t *tg,
                                           const uint32_t *fp, uint32_t sh, uint64_t &any, Bits<C> &bits,
                                           const PreWords<C> *pre) {
  if constexpr (PRE) {
    pass_exact_w<C, ANY, TABLE, NT, OUTK>(pre->w, pre->d, os, m, r, tg, fp, sh, any, bits);
  } else {
    uint32_t w[16 + C / 4], d[C / 4 + 1];
    load_words<16 + C / 4>(w, tw);
    load_words<C / 4 + 1>(d, os.d);
    pass_exact_w<C, ANY, TABLE, NT, OUTK>(w, d, os, m, r, tg, fp, sh, any, bits);
  }
}

template <int C, bool ANY, bool TABLE, int NT, bool PRE>
__device__ __forceinline__ void pass_exact_r(const uint32_t *tw, OutStream os, uint32_t m, uint32_t r, const uint32_t *tg,
                                             const uint32_t *fp, uint32_t sh, uint64_t &any, Bits<C> &bits,
                                             const PreWords<C> *pre) {
  const int k = out_kind(r);
  if (k == 0) pass_exact<C, ANY, TABLE, NT, 0, PRE>(tw, os, m, r, tg, fp, sh, any, bits, pre);
  else if (k == 1) pass_exact<C, ANY, TABLE, NT, 1, PRE>(tw, os, m, r, tg, fp, sh, any, bits, pre);
  else pass_exact<C, ANY, TABLE, NT, 2, PRE>(tw, os, m, r, tg, fp, sh, any, bits, pre);
}

// Destination of a hash dump: the canonical hash of every window whose start
// x = e - m + 1 is a multiple of stride goes to out[x / stride] (x / stride < cap).
struct DumpDst {
  uint64_t *out;
  uint64_t stride;
  uint64_t cap;
};

// kDump: the exact pass's own rolling loop (roll_exact, same out-kind
// specialisation as the test passes), writing canonical states of sampled
// windows instead of testing them.
template <int C, int OUTK>
__device__ __forceinline__ void pass_dump_w(const uint32_t *w, const uint32_t *d, OutStream os, uint32_t m, uint32_t r,
                                            int64_t e0, uint64_t n, const DumpDst &dst) {
  const int64_t x0 = e0 - (int64_t)m + 1;
  // rem = x0 mod stride for the first window (x0 may be negative)
  const int64_t st = (int64_t)dst.stride;
  int64_t rem = x0 % st;
  if (rem < 0) rem += st;
  // slot of the next sampled window at or after x0 (x0 - rem is a multiple of st)
  int64_t slot = (x0 - rem) / st + (rem ? 1 : 0);
  roll_exact<C, OUTK>(w, d, os, m, r, [&](int i, uint64_t s) __attribute__((always_inline)) {
    const int64_t x = x0 + i;
    if (rem == 0) {
      if (x >= 0 && (uint64_t)x + m <= n && (uint64_t)slot < dst.cap) dst.out[slot] = canon(s);
      ++slot;
    }
    rem = (rem + 1 == st) ? 0 : rem + 1;
  });
}

// The dump of one tile for the thread: words from registers (pre) or the LDS tile.
template <int C, bool PRE>
__device__ __forceinline__ void pass_dump(const uint32_t *tw, OutStream os, uint32_t m, uint32_t r, int64_t e0, uint64_t n,
                                          const DumpDst &dst, const PreWords<C> *pre) {
  uint32_t wl[PRE ? 1 : 16 + C / 4], dl[PRE ? 1 : C / 4 + 1];
  const uint32_t *w = wl, *d = dl;
  if constexpr (PRE) {
    w = pre->w;
    d = pre->d;
  } else {
    load_words<16 + C / 4>(wl, tw);
    load_words<C / 4 + 1>(dl, os.d);
  }
  const int k = out_kind(r);
  if (k == 0) pass_dump_w<C, 0>(w, d, os, m, r, e0, n, dst);
  else if (k == 1) pass_dump_w<C, 1>(w, d, os, m, r, e0, n, dst);
  else pass_dump_w<C, 2>(w, d, os, m, r, e0, n, dst);
}

// Runs the test pass of bucket D over the thread's windows: ANY=true ORs the
// wave ballots into any, ANY=false fills the per-thread candidate mask.
// D.shift holds the screen shift in bits 0-7 and the number of list targets
// (1, or up to 4 padded by repetition) in bits 8-15.  PRE: the thread's words
// are already in registers (*pre); else each pass reads them from the tile.
template <int C, bool ANY, int FAM, bool PRE = false>
__device__ __forceinline__ void run_pass(const BucketDesc &D, const uint32_t *tw, OutStream os, uint32_t r,
                                         const uint32_t *fp, uint64_t &any, Bits<C> &bits,
                                         const PreWords<C> *pre = nullptr) {
  const uint32_t sh = D.shift & 0xFFu;
  if constexpr (FAM == kFamScreen1) {
    if (sh == 2) pass_list_screen<C, 2, 1, ANY, PRE>(tw, D.mask, D.tgt, any, bits, pre);
    else if (sh == 4) pass_list_screen<C, 4, 1, ANY, PRE>(tw, D.mask, D.tgt, any, bits, pre);
    else pass_list_screen<C, 8, 1, ANY, PRE>(tw, D.mask, D.tgt, any, bits, pre);
  } else if constexpr (FAM == kFamScreen) {
    if (D.kind == kListScreen) {
      if ((D.shift >> 8) == 1u) {
        if (sh == 2) pass_list_screen<C, 2, 1, ANY, PRE>(tw, D.mask, D.tgt, any, bits, pre);
        else if (sh == 4) pass_list_screen<C, 4, 1, ANY, PRE>(tw, D.mask, D.tgt, any, bits, pre);
        else pass_list_screen<C, 8, 1, ANY, PRE>(tw, D.mask, D.tgt, any, bits, pre);
      } else {
        if (sh == 2) pass_list_screen<C, 2, 4, ANY, PRE>(tw, D.mask, D.tgt, any, bits, pre);
        else if (sh == 4) pass_list_screen<C, 4, 4, ANY, PRE>(tw, D.mask, D.tgt, any, bits, pre);
        else pass_list_screen<C, 8, 4, ANY, PRE>(tw, D.mask, D.tgt, any, bits, pre);
      }
    } else {
      if (sh == 2) pass_table_screen<C, 2, ANY, PRE>(tw, D.mask, fp, D.fp_mask, any, bits, pre);
      else if (sh == 4) pass_table_screen<C, 4, ANY, PRE>(tw, D.mask, fp, D.fp_mask, any, bits, pre);
      else pass_table_screen<C, 8, ANY, PRE>(tw, D.mask, fp, D.fp_mask, any, bits, pre);
    }
  } else {
    // the single-bucket kernel (PRE) runs list buckets only
    if (PRE || D.kind == kListExact) {
      if ((D.shift >> 8) <= 2u) pass_exact_r<C, ANY, false, 2, PRE>(tw, os, D.m, r, D.tgt, fp, D.fp_mask, any, bits, pre);
      else pass_exact_r<C, ANY, false, 4, PRE>(tw, os, D.m, r, D.tgt, fp, D.fp_mask, any, bits, pre);
    } else {
      pass_exact_r<C, ANY, true, 2, PRE>(tw, os, D.m, r, D.tgt, fp, D.fp_mask, any, bits, pre);
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
  wg_barrier();
  if (lane == 63) wsum[wave] = x;
  wg_barrier();
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

// The four bytes ending at *last (LDS, any alignment) in memory order (the
// oldest in the low byte), from the two aligned dwords that hold them.
__device__ __forceinline__ uint32_t raw_word_ending_at(const uint8_t *last) {
  const uint8_t *a = last - 3;
  const uint32_t mis = (uint32_t)(uintptr_t)a & 3u;
  const uint32_t *aw = (const uint32_t *)(a - mis);
  return __builtin_amdgcn_alignbyte(aw[1], aw[0], mis);
}

// The same four bytes as a big-endian word: (last[-3] << 24) | ... | last[0].
__device__ __forceinline__ uint32_t word_ending_at(const uint8_t *last) {
  return __builtin_bswap32(raw_word_ending_at(last));
}

// Exact hash (canonical) of the m <= kStreamM bytes ending at *end (LDS):
// Horner over big-endian words, 2^32 per word (four bytes at a time), the
// oldest word masked to the window's bytes.  The candidate key of exact
// buckets; equal to the value the rolling pass held for that window.
__device__ __forceinline__ uint64_t exact_key(const uint8_t *end, uint32_t m) {
  const uint32_t nw = (m + 3u) >> 2, lead = 4u * nw - m;  // lead: bytes of the oldest word before the window
  uint64_t s = 0;
  for (uint32_t j = nw; j-- > 0;) {
    uint32_t w = word_ending_at(end - 4 * j);
    if (j == nw - 1u && lead) w &= 0xFFFFFFFFu >> (8u * lead);
    s = mul2p32_lazy(s) + w;
  }
  return canon(s);
}

// Shift-add value of four window bytes rw (memory order: the oldest in the
// low byte) with the oldest weighted 2^(3s), ..., the newest 1: one byte dot
// product for s = 2, two for s = 4, the big-endian word for s = 8.
__device__ __forceinline__ uint32_t screen_word(uint32_t rw, uint32_t shift) {
  if (shift == 2) return __builtin_amdgcn_udot4(rw, 0x01041040u, 0u, false);
  if (shift == 4)
    return (__builtin_amdgcn_udot4(rw, 0x00000110u, 0u, false) << 8) + __builtin_amdgcn_udot4(rw, 0x01100000u, 0u, false);
  return __builtin_bswap32(rw);
}

// Shift-add hash of the span = 32/s bytes ending at *end (the value the scan's
// screen pass held for that window end), masked as the group's hash is.
// Four bytes at a time: word j back from the end weighs 2^(4 s j).
__device__ __forceinline__ uint32_t screen_key(const uint8_t *end, uint32_t shift, uint32_t mask) {
  const uint32_t span = 32u / shift, nw = span >> 2;
  uint32_t h = 0;
  for (uint32_t j = nw; j-- > 0;) {
    const uint32_t v = screen_word(raw_word_ending_at(end - 4 * j), shift);
    h = j == nw - 1u ? v : (h << (4 * shift)) + v;  // (one word when shift = 8: no 32-bit shift)
  }
  return h & mask;
}

// Record (slot_inline / slot_run) stored under key in a list bucket's key
// table, read from the instance image in device memory (gimg); 0 if absent.
__device__ __forceinline__ uint64_t key_lookup(const uint8_t *gimg, const BucketDesc &D, uint64_t key) {
  const uint64_t *keys = (const uint64_t *)(gimg + D.ht_off);
  const uint64_t *recs = keys + (D.ht_mask + 1u);
  uint32_t slot = ht_slot(key, D.ht_mask);
  for (uint32_t probe = 0; probe <= D.ht_mask; ++probe) {
    const uint64_t k = keys[slot];
    if (k == key) return recs[slot];
    if (k == kEmptyKey) return 0;
    slot = (slot + 1u) & D.ht_mask;
  }
  return 0;
}

// Record of the 32-bit key h of a table bucket: the cuckoo slot holding h
// (LDS) indexes the per-slot records in device memory.  The load is issued
// without waiting for it: found tells whether h is a key at all (the record
// is then to be dropped), so that the lookups of several candidates overlap.
__device__ __forceinline__ uint64_t table_record(const uint8_t *img, const uint8_t *gimg, const BucketDesc &D,
                                                 uint32_t h, bool &found) {
  const uint32_t *tab = (const uint32_t *)(img + D.fp_off);
  const uint32_t s1 = ck_slot1(h, D.fp_mask), s2 = ck_slot2(h, D.fp_mask);
  const bool in1 = tab[s1] == h, in2 = tab[s2] == h;
  found = in1 || in2;
  return ((const uint64_t *)(gimg + D.ht_off))[in1 ? s1 : s2];
}

// Compares the m bytes ending at *end (LDS tile, any alignment) with the
// pattern at pat (device memory, 4-byte aligned), four bytes per step: the tile
// dwords are realigned with alignbyte and the tail of the last one is masked.
__device__ __forceinline__ bool window_equals(const uint8_t *end, const uint8_t *pat, uint32_t m) {
  const uint8_t *a = end - (m - 1);
  const uint32_t mis = (uint32_t)(uintptr_t)a & 3u;
  const uint32_t *aw = (const uint32_t *)(a - mis);
  const uint32_t *pw = (const uint32_t *)pat;
  uint32_t lo = aw[0];
  for (uint32_t q = 0; 4 * q < m; ++q) {
    const uint32_t hi = aw[q + 1];
    const uint32_t rem = m - 4 * q;
    const uint32_t keep = rem >= 4 ? 0xFFFFFFFFu : ((1u << (8 * rem)) - 1u);
    if ((__builtin_amdgcn_alignbyte(hi, lo, mis) ^ pw[q]) & keep) return false;
    lo = hi;
  }
  return true;
}

// Compares the m <= kFront bytes ending at *end (LDS tile) with a pattern
// whose first 16 bytes are hd (already in registers) and whose bytes are at
// pat (device memory, 4-byte aligned): the first min(m, 16) bytes against hd,
// the rest, if they agree, four bytes per step against pat.
__device__ __forceinline__ bool window_equals_head(const uint8_t *end, const uint32_t (&hd)[4], const uint8_t *pat,
                                                   uint32_t m) {
  const uint8_t *a = end - (m - 1);
  const uint32_t mis = (uint32_t)(uintptr_t)a & 3u;
  const uint32_t *aw = (const uint32_t *)(a - mis);
  uint32_t lo = aw[0], diff = 0;
#pragma unroll
  for (uint32_t q = 0; q < 4; ++q) {
    if (4 * q < m) {
      const uint32_t hi = aw[q + 1];
      const uint32_t rem = m - 4 * q;
      const uint32_t keep = rem >= 4 ? 0xFFFFFFFFu : ((1u << (8 * rem)) - 1u);
      diff |= (__builtin_amdgcn_alignbyte(hi, lo, mis) ^ hd[q]) & keep;
      lo = hi;
    }
  }
  if (diff) return false;
  const uint32_t *pw = (const uint32_t *)pat;
  for (uint32_t q = 4; 4 * q < m; ++q) {
    const uint32_t hi = aw[q + 1];
    const uint32_t rem = m - 4 * q;
    const uint32_t keep = rem >= 4 ? 0xFFFFFFFFu : ((1u << (8 * rem)) - 1u);
    if ((__builtin_amdgcn_alignbyte(hi, lo, mis) ^ pw[q]) & keep) return false;
    lo = hi;
  }
  return true;
}

// Compares the m bytes at a (device memory: the text, any alignment) with the
// pattern at pat (device memory, 4-byte aligned), four bytes per step; reads
// only the text dwords that hold bytes of [a, a + m).  For windows longer than
// the tile's front halo.
__device__ __forceinline__ bool window_equals_global(const uint8_t *a, const uint8_t *pat, uint32_t m) {
  const uint32_t mis = (uint32_t)(uintptr_t)a & 3u;
  const uint32_t *aw = (const uint32_t *)(a - mis);
  const uint32_t *pw = (const uint32_t *)pat;
  const uint32_t nd = (mis + m + 3u) >> 2;  // dwords holding window bytes
  uint32_t lo = aw[0];
  for (uint32_t q = 0; 4 * q < m; ++q) {
    const uint32_t hi = q + 1 < nd ? aw[q + 1] : 0u;  // bytes past the window are masked below
    const uint32_t rem = m - 4 * q;
    const uint32_t keep = rem >= 4 ? 0xFFFFFFFFu : ((1u << (8 * rem)) - 1u);
    if ((__builtin_amdgcn_alignbyte(hi, lo, mis) ^ pw[q]) & keep) return false;
    lo = hi;
  }
  return true;
}

// Whether the pattern referenced by om (om_pack) occurs as the window ending
// at *end (LDS tile; global end index e): the window must start inside the
// text and its bytes must equal the pattern's (the byte comparison of Sec. 3.1
// that follows every hash hit).  Windows that reach beyond the tile's front
// halo (patterns longer than kFront) are compared in the text itself (gtext).
__device__ __forceinline__ bool entry_matches(const uint8_t *gimg, const BucketDesc &D, uint32_t om,
                                              const uint8_t *end, int64_t e, const uint8_t *gtext) {
  const uint32_t m = om_len(om);
  const int64_t x = e - (int64_t)m + 1;
  if (x < 0) return false;
  const uint8_t *pat = gimg + D.pat_off + om_off(om);
  if (m <= kFront) return window_equals(end, pat, m);
  return window_equals_global(gtext + x, pat, m);
}

// Verifies the entries of a plain run record (slot_run) for the candidate
// window ending at *end (global end index e).  Consecutive entries with the
// same pattern bytes (identical patterns under several ids) share one
// comparison.  Returns the number of matching entries; bit i of mask is set
// for a matching entry i < 32 of the run.
__device__ __forceinline__ uint32_t verify_run(const uint8_t *gimg, const BucketDesc &D, uint64_t rec, const uint8_t *end,
                                               int64_t e, const uint8_t *gtext, uint32_t &mask) {
  mask = 0;
  const Entry *ent = (const Entry *)(gimg + D.ent_off);
  const uint32_t first = (uint32_t)rec, cnt = (uint32_t)(rec >> 32);
  uint32_t nh = 0, prev = kNoLink;
  bool prev_ok = false;
  for (uint32_t i = 0; i < cnt; ++i) {
    const uint32_t om = ent[first + i].off_m;
    if (om != prev) {
      prev_ok = entry_matches(gimg, D, om, end, e, gtext);
      prev = om;
    }
    if (prev_ok) {
      ++nh;
      if (i < 32) mask |= 1u << i;
    }
  }
  return nh;
}

// Writes the matching entries of a verified record as hit records
// (pid << 40 | start) at slab[o..], up to cap; o advances over all of them.
// pid_counts (optional): per-pattern hit counters, one increment per hit.
__device__ __forceinline__ void write_hits(const uint8_t *gimg, const BucketDesc &D, uint64_t rec, uint32_t mask,
                                           const uint8_t *end, int64_t e, const uint8_t *gtext, uint64_t *slab,
                                           uint32_t cap, uint32_t &o, unsigned long long *pid_counts) {
  if (rec >> 63) {
    if (mask) {
      const uint32_t om = (uint32_t)rec, pid = (uint32_t)(rec >> 32) & 0xFFFFFFu;
      const uint64_t x = (uint64_t)(e - (int64_t)om_len(om) + 1);
      if (o < cap) slab[o] = ((uint64_t)pid << kPosBits) | x;
      if (pid_counts) atomicAdd(pid_counts + pid, 1ull);
      ++o;
    }
    return;
  }
  const Entry *ent = (const Entry *)(gimg + D.ent_off);
  if (rec_same(rec)) {
    // one pattern under several ids: a hit for each
    if (mask) {
      const uint32_t first = same_first(rec), cnt = same_count(rec);
      const uint64_t x = (uint64_t)(e - (int64_t)om_len((uint32_t)rec) + 1);
      for (uint32_t i = 0; i < cnt; ++i) {
        const uint32_t pid = ent[first + i].pid;
        if (o < cap) slab[o] = ((uint64_t)pid << kPosBits) | x;
        if (pid_counts) atomicAdd(pid_counts + pid, 1ull);
        ++o;
      }
    }
    return;
  }
  const uint32_t first = (uint32_t)rec, cnt = (uint32_t)(rec >> 32);
  for (uint32_t i = 0; i < cnt; ++i) {
    const Entry en = ent[first + i];
    const bool hit = i < 32 ? ((mask >> i) & 1u) != 0 : entry_matches(gimg, D, en.off_m, end, e, gtext);
    if (!hit) continue;
    const uint64_t x = (uint64_t)(e - (int64_t)om_len(en.off_m) + 1);
    if (o < cap) slab[o] = ((uint64_t)en.pid << kPosBits) | x;
    if (pid_counts) atomicAdd(pid_counts + en.pid, 1ull);
    ++o;
  }
}

// ------------------------------------------------------- tile staging (LDS DMA)
// One 16-byte chunk per active lane from device memory straight into LDS:
// lane i's chunk at g lands at dst + 16 i (dst wave-uniform).  Issued in asm
// so that the compiler does not see an LDS write in flight: it would make
// every later LDS read wait for all such loads (vmcnt(0)), the reads of the
// tile being tested included, so that the next tile's loads would no longer
// overlap its test.  Every read of a slot is ordered after that slot's loads
// by the tile pipeline's own waits (wg_barrier_loads).
// (M0 holds the LDS address, placed there by the compiler; the s_nop is the
// wait state required between a write of M0 and the load that uses it.)  The
// loads are non-temporal (nt): the text is read once, and streaming it past
// the caches reads 4 GiB at 6.6 TB/s against 6.1 without the hint.
__device__ __forceinline__ void lds_dma16(const void *g, const uint8_t *dst) {
  const uint32_t m0 = __builtin_amdgcn_readfirstlane(lds_addr(dst));
  __asm__ volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off nt" ::"v"(g), "{m0}"(m0) : "memory");
}

// Issues the loads of one tile into an LDS slot: text bytes [tstart - kFront,
// tstart + W) as 16-byte chunks that the load unit writes straight into LDS
// (no register staging, so the next tile's loads cost no VGPRs while they are
// in flight).  The body is W/1024 whole-wave loads of 1 KiB (lane i: bytes
// 16i..16i+15) dealt round-robin to the waves; the last wave also loads the
// 64-byte front halo with four lanes.  Chunks outside the text read the
// text's first chunk instead: those LDS bytes only feed windows that start
// before the text or end after it, which the edge masks drop.
template <int WG, int C>
__device__ __forceinline__ void dma_tile(uint8_t *slot, const uint8_t *text, uint64_t n, int64_t tstart) {
  constexpr uint32_t W = WG * C, J = W / 1024, NW = WG / 64;
  static_assert(W % 1024 == 0, "a tile is a whole number of 1 KiB wave loads");
  const uint32_t lane = threadIdx.x & 63, wave = uni(threadIdx.x >> 6);
  if (tstart >= (int64_t)kFront && (uint64_t)tstart + W <= n) {
    // interior tile: every chunk is text
    const uint8_t *base = text + tstart + 16u * lane;
    for (uint32_t j = wave; j < J; j += NW)
      lds_dma16(base + 1024u * j, slot + kFront + 1024u * j);
    if (wave == NW - 1 && lane < 4)
      lds_dma16(base - kFront, slot);
    return;
  }
  for (uint32_t j = wave; j < J; j += NW) {
    const uint64_t g = (uint64_t)tstart + 1024u * j + 16u * lane;
    const uint8_t *src = g < n ? text + g : text;
    lds_dma16(src, slot + kFront + 1024u * j);
  }
  if (wave == NW - 1 && lane < 4) {
    const int64_t g = tstart - (int64_t)kFront + 16 * (int64_t)lane;
    const uint8_t *src = g >= 0 ? text + g : text;
    lds_dma16(src, slot);
  }
}

// Candidate phase of one bucket on one tile.  bits holds the thread's
// candidate mask (window i of the thread at bit word_windows-1-(i%32) of word
// i/32).  Windows that start before the text or end after it are dropped, the
// candidates are compacted block-wide into the LDS list in window order, and
// each is checked by one thread: key recomputed, its record (table buckets:
// the cuckoo slot in the LDS image img; list buckets: the key table in the
// device image gimg), byte comparison with every pattern of the record.  Hits
// go to the tile's slab (up to cap records) in window order; tile_hits counts
// them all.  ncand returns the number of candidates (block-uniform).
template <int WG, int C, int Q>
__device__ __forceinline__ void candidate_phase(Bits<C> &bits, const BucketDesc &D, const uint8_t *tile, int64_t tstart,
                                                uint64_t n, int64_t e0, const uint8_t *img, const uint8_t *gimg,
                                                uint16_t *cand,
                                                uint32_t *misc, uint64_t *slab, uint32_t cap, uint32_t &tile_hits,
                                                uint32_t &ncand, const uint8_t *gtext,
                                                unsigned long long *pid_counts, uint64_t rec1 = 0) {
  static_assert(WG * C <= 65536, "window indices of a tile fit the u16 candidate list");
  constexpr uint32_t W = WG * C;
  constexpr int NB = (C + 31) / 32;
  const uint32_t tid = threadIdx.x;
  const uint32_t m = D.m;
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
  const uint32_t cbase = block_excl_scan<WG>(cnt, misc, ncand);

  for (uint32_t r0 = 0; r0 < ncand; r0 += kCandCap) {
    wg_barrier();  // cand list free
    if (cnt) {
      uint32_t idx = cbase;
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        uint32_t bb = bits.b[j];
        while (bb) {
          const uint32_t hb = 31u - __builtin_clz(bb);  // highest bit = earliest window
          const uint32_t i = 32u * j + (uint32_t)word_windows<C>(j) - 1u - hb;
          bb &= ~(1u << hb);
          if (idx >= r0 && idx < r0 + kCandCap) cand[idx - r0] = (uint16_t)(tid * C + i);
          ++idx;
        }
      }
    }
    wg_barrier();
    const uint32_t nc = min(kCandCap, ncand - r0);
    const bool screen = D.kind == kListScreen || D.kind == kTableScreen;
    const bool table = D.kind == kTableScreen || D.kind == kTableExact;
    // The record stored under a candidate's key; the load is left in flight
    // (found: whether the key is in the bucket at all).
    auto record_of = [&](uint32_t ci, const uint8_t *&end, int64_t &e, bool &found)
        __attribute__((always_inline)) -> uint64_t {
      const uint32_t e_rel = cand[ci];
      end = tile + kFront + e_rel;
      e = tstart + (int64_t)e_rel;
      found = true;
      if (rec1) return rec1;  // the bucket has one key: every candidate's record
      const uint64_t key = screen ? (uint64_t)screen_key(end, D.shift & 0xFFu, D.mask) : exact_key(end, m);
      return table ? table_record(img, gimg, D, (uint32_t)key, found) : key_lookup(gimg, D, key);
    };
    // Up to Q candidates per thread, q = ceil(left / WG) of them, contiguous
    // (thread order is candidate order, so the block scan of hit counts keeps
    // the window order).  Three steps, each issuing its loads for all of the
    // thread's candidates before any is waited for: the records; the first 16
    // bytes of the pattern of each record that holds one pattern; the byte
    // comparisons (longer patterns and runs of patterns read the rest then).
    // Waves holding no candidate skip the lookups.  Q is 1 in the exact
    // family (fewer registers: it keeps its occupancy).
    for (uint32_t i0 = 0; i0 < nc; i0 += Q * WG) {
      const uint32_t left = nc - i0;
      const uint32_t q = left >= Q * WG ? Q : (left + WG - 1) / WG;  // uniform, 1..Q
      const uint32_t c0 = i0 + tid * q;
      const bool wave_has = i0 + (tid & ~63u) * q < nc;               // uniform per wave
      uint64_t rec[Q];
      const uint8_t *end[Q];
      int64_t e[Q];
      uint32_t nh[Q], hm[Q];
      bool fnd[Q];
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        rec[j] = 0;
        end[j] = tile;
        e[j] = 0;
        nh[j] = 0;
        hm[j] = 0;
        fnd[j] = false;
      }
      if (wave_has) {
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          if ((uint32_t)j < q) {
            // out-of-range lanes look up the last candidate and drop the result
            const bool v = c0 + j < nc;
            rec[j] = record_of(v ? c0 + j : nc - 1, end[j], e[j], fnd[j]);
            fnd[j] = fnd[j] && v;
          }
        }
        uint32_t hd[Q][4];
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          if (!fnd[j]) rec[j] = 0;
          hd[j][0] = hd[j][1] = hd[j][2] = hd[j][3] = 0;
          if ((uint32_t)j < q && rec_one_pattern(rec[j])) {
            const uint32_t *pw = (const uint32_t *)(gimg + D.pat_off + om_off((uint32_t)rec[j]));
            hd[j][0] = pw[0];
            hd[j][1] = pw[1];
            hd[j][2] = pw[2];
            hd[j][3] = pw[3];
          }
        }
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          if ((uint32_t)j >= q || !rec[j]) continue;
          if (rec_one_pattern(rec[j])) {
            // one pattern (under one id, or under several: a hit per id):
            // starts inside the text, bytes equal (Sec. 3.1)
            const uint32_t om = (uint32_t)rec[j], mj = om_len(om);
            const int64_t x = e[j] - (int64_t)mj + 1;
            const uint8_t *pat = gimg + D.pat_off + om_off(om);
            const bool ok = x >= 0 && (mj <= kFront ? window_equals_head(end[j], hd[j], pat, mj)
                                                     : window_equals_global(gtext + x, pat, mj));
            hm[j] = ok ? 0xFFFFFFFFu : 0u;
            nh[j] = ok ? (rec_same(rec[j]) ? same_count(rec[j]) : 1u) : 0u;
          } else {
            nh[j] = verify_run(gimg, D, rec[j], end[j], e[j], gtext, hm[j]);
          }
        }
      }
      uint32_t mine = 0;
#pragma unroll
      for (int j = 0; j < Q; ++j) mine += nh[j];
      uint32_t nht;
      const uint32_t hb = block_excl_scan<WG>(mine, misc, nht);
      if (mine) {
        uint32_t o = tile_hits + hb;
#pragma unroll
        for (int j = 0; j < Q; ++j)
          if (nh[j]) write_hits(gimg, D, rec[j], hm[j], end[j], e[j], gtext, slab, cap, o, pid_counts);
      }
      tile_hits += nht;
    }
  }
  // nothing of this phase left in flight (a load whose value some path did
  // not use would otherwise make the compiler wait for it, with a count that
  // also covers the next tile's loads, at the next LDS read)
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
}

// A tile with at least this many candidates in a bucket makes the next tile
// of the workgroup skip that bucket's test pass (hits are dense: the mask pass
// runs directly).  Sparse hits (a planted occurrence now and then) keep the
// cheaper test pass.
constexpr uint32_t kDenseCand = 32;

// Bucket descriptor b of the LDS image, as wave-uniform values.
__device__ __forceinline__ BucketDesc read_desc(const uint8_t *img, uint32_t b) {
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
  D.max_m = 0;
  D.pat_off = uni(dp->pat_off);
  D.npat = 0;
  return D;
}

// ------------------------------------------------------------ the scan kernel
//
// LDS: [slot 0][slot 1][cand: kCandCap u16][misc: 64 u32][image: img_cap]
template <int WG, int C, int FAM>
__global__ __launch_bounds__(WG) void scan_kernel(ScanParams p) {
  constexpr uint32_t W = WG * C;
  constexpr uint32_t TILE_LDS = (kFront + W + 16 + 15) & ~15u;  // one slot
  constexpr int NB = (C + 31) / 32;
  extern __shared__ __align__(16) uint8_t lds[];
  uint16_t *cand = (uint16_t *)(lds + 2 * TILE_LDS);
  uint32_t *misc = (uint32_t *)(cand + kCandCap);  // [0,16) scan sums, [16,48) any flags, [48] queue
  uint8_t *img = (uint8_t *)(misc + 64);

  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint32_t cur_inst = kNoLink;
  uint64_t static_item = blockIdx.x;
  uint32_t flag_parity = 0;
  uint32_t dense_mask = 0;  // buckets whose last tile had candidates
  const uint64_t nitems = p.nitems_dev ? min(p.nitems, (uint64_t)*p.nitems_dev) : p.nitems;

  // Next work item (uniform across the workgroup).  With a queue, thread 0
  // pops and the value is read back after the barrier that follows.
  auto pop = [&]() -> uint64_t {
    if (p.queue) {
      wg_barrier();
      if (tid == 0) misc[48] = atomicAdd(p.queue, 1u);
      wg_barrier();
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
  // Two LDS slots: tile k is processed in one while the loads of tile k+1
  // land in the other.
  uint32_t slot = 0;
  const uint8_t *gimg = nullptr;  // current instance image in device memory
  uint64_t item = pop();
  Item cur;
  if (item < nitems) {
    cur = locate(item);
    dma_tile<WG, C>(lds, cur.text, cur.n, cur.tstart);
  }
  while (item < nitems) {
    const uint64_t next = pop();
    const bool have_next = next < nitems;
    Item nx;
    if (have_next) nx = locate(next);
    // this tile has landed, and every wave is done with the other slot
    wg_barrier_loads();
    uint8_t *tile = lds + slot * TILE_LDS;
    if (cur.inst != cur_inst) {
      // the image's leading part goes to LDS; the rest is read in place
      gimg = p.blob + p.inst[cur.inst].img_off;
      const uint4 *src = (const uint4 *)gimg;
      uint4 *dst = (uint4 *)img;
      const uint32_t nq = p.inst[cur.inst].lds_bytes / 16u;
      for (uint32_t q = tid; q < nq; q += WG) dst[q] = src[q];
      cur_inst = cur.inst;
      wg_barrier();
    }
    const uint64_t gt = cur.gt;
    const uint64_t n = cur.n;
    const int64_t tstart = cur.tstart;
    uint64_t *slab = nullptr;
    if (p.out) slab = p.direct ? (p.out + p.tile_offsets[gt]) : (p.out + (gt - p.tile0) * (uint64_t)p.slab_cap);
    const uint32_t cap = p.direct ? 0xFFFFFFFFu : p.slab_cap;
    // Everything this tile reads from memory into registers is there before
    // the next tile's loads are issued (the compiler would otherwise wait for
    // a late load with a count that also covers those loads).
    __asm__ volatile("" ::"v"(slab), "v"(n), "v"(tstart), "v"(gt), "v"(gimg) : "memory");
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    if (have_next) dma_tile<WG, C>(lds + (slot ^ 1u) * TILE_LDS, nx.text, nx.n, nx.tstart);

    // this thread's bytes: 64 before its first window end, then C
    const uint32_t *tw = (const uint32_t *)(tile + kFront + tid * C - 64);
    const uint8_t *mine = tile + kFront + tid * C;  // LDS byte of my first window end
    const int64_t e0 = tstart + (int64_t)(tid * C); // global end index of my first window

    const ImageHeader *H = (const ImageHeader *)img;
    const uint32_t nb = uni(H->nbuckets);
    uint32_t tile_hits = 0;

    // Buckets go in chunks of 32: the test pass of every bucket of the chunk
    // first (one flag bit per bucket and wave), one barrier, then the mask
    // pass and candidate phase of the buckets whose tile had a candidate.
    for (uint32_t b0 = 0; b0 < nb; b0 += 32) {
      const uint32_t nbc = min(32u, nb - b0);
      uint32_t wave_bits = 0, need = 0;
      for (uint32_t bi = 0; bi < nbc; ++bi) {
        const uint32_t b = b0 + bi;
        const BucketDesc D = read_desc(img, b);
        const uint32_t m = D.m;
        const uint32_t r = (8u * m) % 61u;
        const OutStream os = out_stream(mine, m);
        if constexpr (FAM == kFamExact) {
          if (D.kind == kDump) {
            pass_dump<C, false>(tw, os, m, r, e0, n, DumpDst{p.dump_out, p.dump_stride, p.dump_cap}, nullptr);
            continue;
          }
        }
        // skipped while the bucket's previous tile had candidates (dense
        // hits): the mask pass and its block scan decide then
        if (b < 32 && ((dense_mask >> b) & 1u)) {
          need |= 1u << bi;
          continue;
        }
        uint64_t any = 0;
        Bits<C> nob;
        run_pass<C, true, FAM>(D, tw, os, r, (const uint32_t *)(img + D.fp_off), any, nob);
        if (any) wave_bits |= 1u << bi;
      }
      uint32_t *flags = misc + 16 + 16 * flag_parity;
      flag_parity ^= 1u;
      if (lane == 0) flags[wave] = wave_bits;
      wg_barrier();
#pragma unroll
      for (int i = 0; i < WG / 64; ++i) need |= flags[i];
      need = uni(need);
      while (need) {
        const uint32_t bi = __builtin_ctz(need);
        need &= need - 1u;
        const uint32_t b = b0 + bi;
        const BucketDesc D = read_desc(img, b);
        const uint32_t m = D.m;
        const uint32_t r = (8u * m) % 61u;
        const OutStream os = out_stream(mine, m);
        Bits<C> bits;
#pragma unroll
        for (int j = 0; j < NB; ++j) bits.b[j] = 0;
        uint64_t dummy = 0;
        run_pass<C, false, FAM>(D, tw, os, r, (const uint32_t *)(img + D.fp_off), dummy, bits);
        uint32_t ncand;
        candidate_phase<WG, C, FAM == kFamExact ? 1 : kCandCap / WG>(bits, D, tile, tstart, n, e0, img, gimg, cand,
                                                                     misc, slab, cap,
                                                     tile_hits, ncand,
                               cur.text, p.direct ? nullptr : p.pid_counts);
        if (b < 32) dense_mask = ncand >= kDenseCand ? (dense_mask | (1u << b)) : (dense_mask & ~(1u << b));
      }
    }

    if (tid == 0 && !p.direct) {
      p.tile_counts[gt] = tile_hits;
      if (tile_hits) {
        atomicAdd(p.total, (unsigned long long)tile_hits);
        if (p.blk_sums) atomicAdd(p.blk_sums + (gt >> kTileSumLog2), (unsigned long long)tile_hits);
      }
      if (tile_hits > p.slab_cap) {
        const uint32_t o = atomicAdd(p.ovf_count, 1u);
        p.ovf_list[o] = gt;
      }
    }
    item = next;
    cur = nx;
    slot ^= 1u;
  }
}

// ------------------------------------------------- single-bucket scan kernel
// The same scan for the most common plan shape: one text and one bucket whose
// set fits in registers (up to 4 targets: one pattern, or a few patterns of
// similar length).  The bucket descriptor and the text come as kernel
// arguments, tiles are strided statically over the persistent grid, and there
// is no image staging, work list or instance lookup, so a tile costs little
// beyond its hash pass.  Count mode only (hits into per-tile slabs); a tile
// whose slab overflows is rescanned by the general kernel.
//
// Tile t+1 loads into the other slot while tile t is tested: the thread's
// words of tile t are read into registers first (out of the compiler's sight,
// so that it does not wait for the new loads), then tile t+1's loads are
// issued, then the test runs on registers only.
//
// LDS: [slot 0][slot 1][cand: kCandCap u16][misc: 64 u32]
template <int WG, int C, int FAM>
__global__ __launch_bounds__(WG) void scan_list_kernel(ListParams p) {
  constexpr uint32_t W = WG * C;
  constexpr uint32_t TILE_LDS = (kFront + W + 16 + 15) & ~15u;
  constexpr int NB = (C + 31) / 32;
  extern __shared__ __align__(16) uint8_t lds[];
  uint16_t *cand = (uint16_t *)(lds + 2 * TILE_LDS);
  uint32_t *misc = (uint32_t *)(cand + kCandCap);
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const BucketDesc D = p.D;
  const uint32_t m = D.m;
  const uint32_t r = p.rot;
  uint32_t slot = 0, flag_parity = 0;
  bool dense = false;
  uint64_t t = blockIdx.x;
  if (t < p.ntiles) dma_tile<WG, C>(lds, p.text, p.n, (int64_t)(t * W));
  while (t < p.ntiles) {
    const uint64_t nt = t + gridDim.x;
    wg_barrier_loads();  // tile t has landed; every wave is done with the other slot
    const uint8_t *tile = lds + slot * TILE_LDS;
    const int64_t tstart = (int64_t)(t * W);
    const uint32_t *tw = (const uint32_t *)(tile + kFront + tid * C - 64);
    const OutStream os = out_stream(tile + kFront + tid * C, m);
    PreWords<C> pre;
    load_words<16 + C / 4>(pre.w, tw);
    if constexpr (FAM == kFamExact) load_words<C / 4 + 1>(pre.d, os.d);
    if (nt < p.ntiles) dma_tile<WG, C>(lds + (slot ^ 1u) * TILE_LDS, p.text, p.n, (int64_t)(nt * W));
    const int64_t e0 = tstart + (int64_t)(tid * C);
    if constexpr (FAM == kFamExact) {
      if (D.kind == kDump) {
        // hash dump: this kernel's own rolling loop over the words read above
        pass_dump<C, true>(tw, os, m, r, e0, p.n, DumpDst{p.dump_out, p.dump_stride, p.dump_cap}, &pre);
        t = nt;
        slot ^= 1u;
        continue;
      }
    }
    uint32_t tile_hits = 0;
    bool run2 = dense;
    if (!dense) {
      uint64_t any = 0;
      Bits<C> nob;
      run_pass<C, true, FAM, true>(D, tw, os, r, nullptr, any, nob, &pre);
      uint32_t *flags = misc + 16 + 16 * flag_parity;
      flag_parity ^= 1u;
      if (lane == 0) flags[wave] = any != 0;
      wg_barrier();
      uint32_t blk_any = 0;
#pragma unroll
      for (int i = 0; i < WG / 64; ++i) blk_any |= flags[i];
      run2 = blk_any != 0;
    }
    if (run2) {
      Bits<C> bits;
#pragma unroll
      for (int j = 0; j < NB; ++j) bits.b[j] = 0;
      uint64_t dummy = 0;
      run_pass<C, false, FAM, true>(D, tw, os, r, nullptr, dummy, bits, &pre);
      uint32_t ncand;
      candidate_phase<WG, C, FAM == kFamExact ? 1 : 2>(bits, D, tile, tstart, p.n, e0, nullptr, p.gimg, cand, misc,
                             p.out + t * (uint64_t)p.slab_cap, p.slab_cap, tile_hits, ncand, p.text, p.pid_counts,
                             p.rec1);
      dense = ncand >= kDenseCand;
    }
    if (tid == 0) {
      p.tile_counts[t] = tile_hits;
      if (tile_hits) {
        atomicAdd(p.total, (unsigned long long)tile_hits);
        if (p.blk_sums) atomicAdd(p.blk_sums + (t >> kTileSumLog2), (unsigned long long)tile_hits);
      }
      if (tile_hits > p.slab_cap) {
        const uint32_t o = atomicAdd(p.ovf_count, 1u);
        p.ovf_list[o] = t;
      }
    }
    t = nt;
    slot ^= 1u;
  }
}

// ------------------------------------------------------------------ launchers
template <int WG, int C>
constexpr uint32_t list_lds_bytes_t() {
  return 2 * ((kFront + WG * C + 16 + 15) & ~15u) + kCandCap * 2 + 64 * 4;
}

template <int WG, int C, int FAM>
static hipError_t launch_scan_t(const ScanParams &p, uint32_t grid, uint32_t lds_bytes, hipStream_t s) {
  // the dynamic LDS limit was raised by prepare_scan_kernels() at context creation
  hipLaunchKernelGGL((scan_kernel<WG, C, FAM>), dim3(grid), dim3(WG), lds_bytes, s, p);
  return hipGetLastError();
}

template <int WG, int C, int FAM>
static hipError_t launch_list_t(const ListParams &p, uint32_t grid, hipStream_t s) {
  constexpr uint32_t lds = list_lds_bytes_t<WG, C>();
  hipLaunchKernelGGL((scan_list_kernel<WG, C, FAM>), dim3(grid), dim3(WG), lds, s, p);
  return hipGetLastError();
}

// Geometry CFG of kTileCfgs as template arguments.
template <int CFG>
struct Geom {
  static constexpr int WG = kTileCfgs[CFG].wg, C = kTileCfgs[CFG].c;
};

template <int FAM, int CFG>
hipError_t ScanGeom<FAM, CFG>::launch(const ScanParams &p, uint32_t grid, uint32_t lds_bytes, hipStream_t s) {
  return launch_scan_t<Geom<CFG>::WG, Geom<CFG>::C, FAM>(p, grid, lds_bytes, s);
}

template <int FAM, int CFG>
hipError_t ScanGeom<FAM, CFG>::occupancy(uint32_t lds_bytes, int *blocks) {
  constexpr int WG = Geom<CFG>::WG, C = Geom<CFG>::C;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void *)scan_kernel<WG, C, FAM>, WG, lds_bytes);
}

template <int FAM, int CFG>
hipError_t ScanGeom<FAM, CFG>::list(const ListParams *p, uint32_t grid, hipStream_t s, int *blocks) {
  constexpr int WG = Geom<CFG>::WG, C = Geom<CFG>::C;
  if (p) return launch_list_t<WG, C, FAM>(*p, grid, s);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, (const void *)scan_list_kernel<WG, C, FAM>, WG,
                                                      list_lds_bytes_t<WG, C>());
}

template <int FAM, int CFG>
hipError_t ScanGeom<FAM, CFG>::prepare() {
  return hipFuncSetAttribute((const void *)scan_kernel<Geom<CFG>::WG, Geom<CFG>::C, FAM>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template <int FAM, int CFG>
hipError_t ScanGeom<FAM, CFG>::list_prepare() {
  return hipFuncSetAttribute((const void *)scan_list_kernel<Geom<CFG>::WG, Geom<CFG>::C, FAM>,
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

// Explicit instantiation of the general kernel's launchers (X = launch) or
// the single-bucket kernel's (X = list) for family FAM and geometry CFG.
#define RK_INSTANTIATE_SCAN(FAM, CFG)                                                                     \
  template hipError_t ScanGeom<FAM, CFG>::launch(const ScanParams &, uint32_t, uint32_t, hipStream_t); \
  template hipError_t ScanGeom<FAM, CFG>::occupancy(uint32_t, int *);                                   \
  template hipError_t ScanGeom<FAM, CFG>::prepare();
#define RK_INSTANTIATE_LIST(FAM, CFG)                                                                    \
  template hipError_t ScanGeom<FAM, CFG>::list(const ListParams *, uint32_t, hipStream_t, int *);      \
  template hipError_t ScanGeom<FAM, CFG>::list_prepare();

}  // namespace rk
