// Internal layouts shared by the host runtime and the HIP kernels of librk.
//
// Text windows are identified by their END byte e (window = T[e-m+1 .. e]):
// a tile owns the windows whose last byte falls inside it, so every thread
// ingests its own bytes at static register positions and the (m-1)-byte
// halo sits in front of the tile.  Start position x = e - m + 1.
#pragma once
#include <stdint.h>

namespace rk {

constexpr uint64_t kQ = (1ull << 61) - 1;  // Mersenne modulus 2^61 - 1
constexpr uint32_t kFront = 64;            // halo bytes kept in front of a tile (= kStreamM)
constexpr uint32_t kStreamM = 64;          // longest window hashed by a rolling stream; longer patterns are
                                           // keyed by their last kStreamM bytes
constexpr uint32_t kPosBits = 40;          // hit record = pid << 40 | start position
constexpr uint64_t kPosMask = (1ull << kPosBits) - 1;
constexpr uint32_t kCandCap = 1024;        // candidate slots in LDS per workgroup (window index in the tile, u16)
constexpr uint32_t kMaxWaves = 16;
constexpr uint32_t kNoLink = 0xFFFFFFFFu;
constexpr uint64_t kEmptyKey = ~0ull;      // empty exact-table slot (no canonical hash is >= q)

// Screen/test variants of one bucket (one pattern length inside one instance).
enum BucketKind : uint32_t {
  kListScreen = 0,   // screen mode: shift-add hash compared with up to 4 targets
  kTableScreen = 1,  // screen mode: shift-add hash probed in the LDS cuckoo table
  kListExact = 2,    // exact mode: lazy 61-bit state compared with up to 4 lazy targets
  kTableExact = 3,   // exact mode: low word of the canonical 61-bit hash probed in the cuckoo table
  kDump = 4,         // exact rolling state written out for sampled windows (no patterns)
};

// Group descriptor as laid out in an instance image (64 bytes).  A group is a
// set of patterns tested with one hash stream: one length class in exact mode
// (keyed on its shortest length), one screen-hash span in screen mode.
struct BucketDesc {
  uint32_t m;          // the group's shortest length: the window its exact stream hashes
  uint32_t kind;       // BucketKind
  uint32_t shift;      // screen groups: shift s in bits 0-7, list target count (1 or 4) in bits 8-15
  uint32_t mask;       // screen-hash mask (all ones unless m < 4 with s = 8)
  uint32_t tgt[4];     // list kinds: targets (padded by repetition)
  uint32_t fp_off;     // table kinds: image offset of the cuckoo table (u32 keys; LDS part)
  uint32_t fp_mask;    // table kinds: 32 - log2(table slots), the slot shift of ck_slot1/2
  uint32_t ht_off;     // list kinds: key table, u64 keys[ht_mask+1] then u64 records[ht_mask+1];
                       // table kinds: u64 records[ht_mask+1], one per cuckoo slot
  uint32_t ht_mask;    // key-table (list) or cuckoo-table (table) slots - 1
  uint32_t ent_off;    // Entry[npat], sorted by (key, length, pattern id)
  uint32_t max_m;      // longest pattern in the group
  uint32_t pat_off;    // pattern bytes; Entry::off_m low 24 bits are relative to this
  uint32_t npat;       // patterns in this group
};
static_assert(sizeof(BucketDesc) == 64, "bucket descriptor is 64 bytes");

// One pattern of a group (16 bytes).
struct Entry {
  uint64_t hx;     // exact hash of the pattern, canonical
  uint32_t pid;    // global pattern id
  uint32_t off_m;  // om_pack(byte offset of the pattern, length)
};
static_assert(sizeof(Entry) == 16, "entry is 16 bytes");

// Pattern reference of an entry: byte offset in its group's pattern block
// (bits 0-21, so a group holds at most 4 MiB of pattern bytes) and length - 1
// (bits 22-31, lengths 1..1024).
constexpr uint32_t kOmOffBits = 22;
constexpr uint32_t kGroupPatBytes = 1u << kOmOffBits;
__host__ __device__ inline uint32_t om_pack(uint32_t off, uint32_t m) { return off | ((m - 1u) << kOmOffBits); }
__host__ __device__ inline uint32_t om_len(uint32_t om) { return (om >> kOmOffBits) + 1u; }
__host__ __device__ inline uint32_t om_off(uint32_t om) { return om & (kGroupPatBytes - 1u); }

// Record of a key (list kinds: in the key table; table kinds: per cuckoo
// slot): the run of entries with that key, or the single entry inline.
//   bit 63 set : one entry, pattern id in bits 32..55, off_m in bits 0..31
//   bits 63-62 = 01: a run of identical patterns (one pattern under several
//                ids): count - 1 in bits 54..61, first entry in bits 32..53,
//                their shared off_m in bits 0..31
//   bits 63-62 = 00: count in bits 32..61 (0: no entry), first entry in bits 0..31
__host__ __device__ inline uint64_t slot_inline(uint32_t pid, uint32_t off_m) {
  return (1ull << 63) | ((uint64_t)pid << 32) | off_m;
}
__host__ __device__ inline uint64_t slot_run(uint32_t first, uint32_t count) {
  return ((uint64_t)count << 32) | first;
}
constexpr uint32_t kSameMaxCount = 256, kSameMaxFirst = 1u << 22;
__host__ __device__ inline uint64_t slot_same(uint32_t first, uint32_t count, uint32_t off_m) {
  return (1ull << 62) | ((uint64_t)(count - 1u) << 54) | ((uint64_t)first << 32) | off_m;
}
__host__ __device__ inline bool rec_one_pattern(uint64_t rec) { return (rec >> 62) != 0; }  // inline or identical run
__host__ __device__ inline bool rec_same(uint64_t rec) { return (rec >> 62) == 1u; }
__host__ __device__ inline uint32_t same_count(uint64_t rec) { return (uint32_t)((rec >> 54) & 0xFFu) + 1u; }
__host__ __device__ inline uint32_t same_first(uint64_t rec) { return (uint32_t)(rec >> 32) & (kSameMaxFirst - 1u); }

// Slot of a key in a group's key table (the host builds it, the kernel probes it).
__host__ __device__ inline uint32_t ht_slot(uint64_t key, uint32_t mask) {
  return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 40) & mask;
}

// Two slots of a 32-bit key in a cuckoo table of 2^(32-sh) slots (built on
// the host, probed by the kernel): multiplicative mixes of the key's low and
// high 24 bits (each a 24 x 24-bit product, one full-rate multiply on gfx950).
__host__ __device__ inline uint32_t ck_slot1(uint32_t h, uint32_t sh) { return ((h & 0xFFFFFFu) * 0x9E3779u) >> sh; }
__host__ __device__ inline uint32_t ck_slot2(uint32_t h, uint32_t sh) { return ((h >> 8) * 0xC2B2AFu) >> sh; }
constexpr uint32_t kMaxTableBits = 13;  // largest cuckoo table: 8192 slots, 32 KiB of LDS

// Header at the start of an instance image (16 bytes), followed by nb
// descriptors, the parts staged in LDS and the parts read from device memory.
struct ImageHeader {
  uint32_t nbuckets;
  uint32_t bytes;      // total image bytes (multiple of 16)
  uint32_t max_m;
  uint32_t lds_bytes;  // leading bytes staged in LDS (header, descriptors, cuckoo tables)
};

// One instance of a scan job (48 bytes).
struct InstDesc {
  const uint8_t *text; // 16-byte aligned
  uint64_t n;
  uint64_t tile_base;  // global id of this instance's tile 0
  uint64_t ntiles;
  uint32_t img_off;    // byte offset of the instance image in the plan blob (16-aligned)
  uint32_t lds_bytes;  // leading image bytes the scan stages in LDS
  uint64_t pad;
};
static_assert(sizeof(InstDesc) == 48, "instance descriptor is 48 bytes");

// The count pass adds each tile's hits to its block of 2^kTileSumLog2 tiles
// (the blocks of the collect's prefix sum of the tile counts, which then
// starts from these sums).
constexpr uint32_t kTileSumLog2 = 12;

// Kernel parameters of the scan (passed by value).
struct ScanParams {
  const InstDesc *inst;
  uint32_t ninst;
  uint32_t img_cap;           // LDS bytes reserved for an instance image
  const uint8_t *blob;        // instance images
  const uint64_t *items;      // item -> global tile id (nullptr: identity)
  uint64_t nitems;
  const uint32_t *nitems_dev; // optional device-side bound on nitems (rescan list length)
  uint32_t *tile_counts;      // hits per global tile
  uint64_t *out;              // count mode: slabs [tile][slab_cap]; direct mode: compact array
  const uint64_t *tile_offsets; // direct mode: first output slot of each tile
  uint32_t slab_cap;
  uint32_t direct;            // 1: rescan writing every hit at tile_offsets[tile]
  unsigned long long *total;  // count mode: hits over all tiles
  uint32_t *ovf_count;        // count mode: number of tiles with more hits than slab_cap
  uint64_t *ovf_list;         // count mode: those tiles' global ids
  uint32_t *queue;            // atomic work-queue cursor (nullptr: static striding)
  uint32_t grab;              // items taken per queue pop
  uint64_t *dump_out;         // kDump buckets: destination of sampled hashes
  uint64_t dump_stride;
  uint64_t dump_cap;
  unsigned long long *pid_counts; // count mode, optional: hits per global pattern id
  uint64_t tile0;             // count mode: global id of the first tile of out's slabs
  unsigned long long *blk_sums; // count mode, optional: hits per 2^kTileSumLog2 global tiles
};

// Kernel parameters of the single-bucket scan (one text, one bucket whose set
// sits in registers; count mode).
struct ListParams {
  const uint8_t *text;        // 16-byte aligned
  uint64_t n;
  uint64_t ntiles;
  const uint8_t *gimg;        // the instance image in device memory (verification tables)
  BucketDesc D;               // the bucket (offsets relative to gimg)
  uint32_t rot;               // 8 m mod 61
  uint32_t slab_cap;
  uint64_t rec1;              // record of the bucket's key if it has exactly one (else 0: look it up)
  uint32_t *tile_counts;
  uint64_t *out;              // slabs [tile][slab_cap]
  unsigned long long *total;
  uint32_t *ovf_count;
  uint64_t *ovf_list;
  uint64_t *dump_out;         // kDump bucket: destination of sampled hashes (no counts then)
  uint64_t dump_stride;
  uint64_t dump_cap;
  unsigned long long *pid_counts; // optional: hits per pattern id
  unsigned long long *blk_sums; // optional: hits per 2^kTileSumLog2 tiles
};

// Host-side geometry table (workgroup size, windows per thread).
struct TileCfg {
  uint32_t wg;
  uint32_t c;
};
constexpr int kNumTileCfg = 4;
constexpr TileCfg kTileCfgs[kNumTileCfg] = {{256, 68}, {256, 132}, {512, 68}, {256, 36}};

// Kernel families: each scan kernel is compiled for the bucket kinds one plan
// can hold, so that a single-pattern search does not pay the register budget
// of the multi-pattern and exact variants.
enum Family : int {
  kFamScreen1 = 0,  // list screen with one target per bucket
  kFamScreen = 1,   // every screen kind
  kFamExact = 2,    // every exact kind and the hash dump
};

}  // namespace rk
