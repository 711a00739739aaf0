// Host-side objects of librk (context, plan, scratch layout) and the launch
// functions exported by the device translation unit.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/rk.h"
#include "rk_internal.h"

namespace rk {

constexpr uint32_t kImgLimit = 64 * 1024;  // largest instance image staged in LDS

struct ProfEvent {
  hipEvent_t a, b;
  int kind;  // 0 scan, 1 rescan, 2 collect
};

struct CountMemo {
  const void *scratch = nullptr;
  const rk_plan *plan = nullptr;
  uint64_t n = 0;
  uint64_t total = 0;
  uint32_t overflow = 0xFFFFFFFFu;  // tiles whose hits did not fit their slab (unknown: all ones)
};

// Pattern-length class of a group (the m-bucket of batch work queues), by
// the length its stream hashes: 0: 1-3, 1: 4-7, 2: 8-15, 3: 16-31, 4: 32-64.
constexpr int kNumMClass = 5;
inline int m_class(uint32_t m) { return m < 4 ? 0 : m < 8 ? 1 : m < 16 ? 2 : m < 32 ? 3 : 4; }
// Pattern-count class of an image: 0: one pattern, 1: 2-4 (register
// targets), 2: 5-64, 3: more.
constexpr int kNumKClass = 4;
inline int k_class(uint32_t k) { return k <= 1 ? 0 : k <= 4 ? 1 : k <= 64 ? 2 : 3; }
constexpr int kMaxParts = kNumTileCfg;  // one persistent launch per scan geometry

struct VInst {
  uint32_t src;       // real instance index
  uint32_t img_off;   // in the plan blob
  uint32_t img_bytes;
  uint32_t lds_bytes;  // leading bytes staged in LDS
  uint32_t nbuckets = 0;
  uint32_t max_m = 0;
  uint32_t npat = 0;   // patterns in the image
  int cfg = 0;         // scan geometry
  bool only_one_list = true;  // every bucket is a list screen with one target
};

// The virtual instances of a plan that share one scan geometry, scanned by
// one persistent launch (a single-text plan has one part).
struct Part {
  int cfg = 0;
  int fam = kFamScreen1;
  uint32_t img_cap = 0;            // LDS bytes reserved for an image
  uint32_t inst0 = 0, ninst = 0;   // its instance descriptors (batch: in inst_dev)
  uint64_t item0 = 0, nitems = 0;  // its work-queue entries in items_dev (batch)
  uint64_t tile0 = 0, ntiles = 0;  // its tiles in the plan's tile numbering (batch)
};

struct RealInst {
  const uint8_t *text;
  uint64_t n;
  uint32_t pid_base;
  uint32_t k;
};

}  // namespace rk

struct rk_ctx {
  int device = 0;
  int num_cu = 0;
  std::string arch;
  std::string err;
  uint32_t slab_cap = 0;
  int tile_cfg = -1;
  uint32_t grid = 0;
  bool profile = false;
  int queue = -1;
  uint64_t *pinned = nullptr;  // 4 KiB of pinned host memory for small transfers
  hipStream_t aux = nullptr;   // the context's own non-blocking stream (plan uploads)
  std::vector<uint8_t> upload; // staging for instance descriptors
  std::vector<rk::ProfEvent> prof_events, free_events;
  int tune[3][RK_MAX_M + 1];
  uint8_t tune_measured[3][RK_MAX_M + 1] = {};
  int tune_b[3][rk::kNumMClass][rk::kNumKClass];  // batch buckets: geometry per (mode, m-class, k-class)
  // batch buckets: tuned time per MiB of text for each geometry (< 0: not measured)
  double tune_bms[3][rk::kNumMClass][rk::kNumKClass][rk::kNumTileCfg];
  rk::CountMemo memo[16];
  uint32_t memo_next = 0;
  void *dump_dev = nullptr;    // device copy of the dump image
  void *static_scratch = nullptr;  // this device's copy of the static scratch array (rk_search_static)
};

struct rk_plan {
  int device = 0;
  int mode = RK_MODE_SCREEN;
  bool batch = false;
  int cfg = 0;
  int fam = rk::kFamScreen1;
  uint32_t k_total = 0;
  uint32_t img_cap = 0;       // LDS bytes reserved for images (max image size)
  bool list1 = false;         // one text, one bucket with register targets: single-bucket kernel
  rk::BucketDesc list_desc;   // that bucket
  uint64_t list_rec1 = 0;     // its key's record when it has a single key
  uint64_t text_bytes = 0;
  uint32_t max_m = 0;         // longest pattern
  std::vector<rk::RealInst> insts;
  std::vector<rk::VInst> vinsts;
  void *dev = nullptr;        // one device allocation: blob | instance descs | items
  uint8_t *blob_dev = nullptr;
  rk::InstDesc *inst_dev = nullptr;  // batch: fixed descriptors (sorted by tile_base)
  uint64_t *items_dev = nullptr;     // batch: queue order of global tile ids, part by part
  uint64_t total_tiles = 0;          // batch
  uint64_t nitems = 0;               // batch
  std::vector<rk::Part> parts;       // one persistent launch each
};

namespace rk {

// One part of a count or collect pass as laid out in scratch.
struct PartRun {
  uint64_t tile0 = 0, ntiles = 0;  // tiles of the part in the pass's numbering
  uint32_t W = 0;                  // tile bytes
  uint32_t S = 0;                  // slab slots per tile
  uint64_t slabs = 0;              // scratch offset of the part's slabs [tile][S]
};

// Scratch of a pass: counters (total at 0, per-part overflow counts at 8 + 4p,
// per-part queue cursors at 48 + 4p), instance descriptors (single plans),
// per-tile counts, offsets and overflow lists, scan partials, slabs.
struct Layout {
  uint64_t T = 0;      // tiles over all parts
  uint64_t T1 = 0;     // tiles per virtual instance (single plans)
  std::vector<PartRun> parts;
  uint64_t ctr = 0, inst = 0, counts = 0, offsets = 0, ovf = 0, total = 0;
  uint64_t bsum = 0, nbsum = 0;  // the tiles' block sums (u64, nbsum entries) right after the 64 counter words
};
constexpr uint32_t kCtrOvf = 8, kCtrQueue = 48;
// Tiles that overflowed their slabs, summed over parts, from the first 64
// counter bytes.
inline uint32_t ovf_total(const uint64_t *ctr) {
  const uint32_t *w = (const uint32_t *)ctr;
  uint32_t t = 0;
  for (int p = 0; p < kMaxParts; ++p) t += w[kCtrOvf / 4 + p];
  return t;
}

rk_status set_err(rk_ctx *ctx, rk_status st, const char *fmt, ...);
rk_status hip_err(rk_ctx *ctx, hipError_t e, const char *what);
inline rk_status hip_err_or_ok(rk_ctx *ctx, hipError_t e) {
  return e == hipSuccess ? RK_OK : hip_err(ctx, e, "profiling event");
}
uint64_t host_hash(const uint8_t *p, uint64_t m);
uint32_t screen_shift(uint32_t m);
uint32_t screen_hash(const uint8_t *p, uint32_t m);

rk_status plan_build(rk_ctx *ctx, const rk_instance *inst, uint32_t count, int mode, bool batch, rk_plan **out);
rk_status make_layout(rk_ctx *ctx, const rk_plan *plan, uint64_t n, Layout &L);
uint64_t work_bytes_for(const rk_plan *plan, uint64_t total);
rk_status count_enqueue(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text, uint64_t n, void *scratch,
                        uint64_t scratch_bytes, uint64_t *counts, hipStream_t s);
rk_status count_finish(rk_ctx *ctx, const rk_plan *plan, void *scratch, hipStream_t s, uint64_t *total);
rk_status collect_enqueue(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text, uint64_t n, void *scratch,
                          uint64_t scratch_bytes, void *work, uint64_t work_bytes, uint64_t *offsets,
                          uint64_t *positions, uint64_t capacity, hipStream_t s);
// text: the counted text (single-text plans: a rescan of overflowed tiles
// reads it; batch plans: null)
rk_status collect_enqueue_known(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text, uint64_t n, void *scratch,
                                uint64_t scratch_bytes, void *work, uint64_t work_bytes, uint64_t *offsets,
                                uint64_t *positions, uint64_t capacity, uint64_t total, uint32_t overflow,
                                hipStream_t s);
rk_status plan_build_host(rk_ctx *ctx, const rk_instance *inst, uint32_t count, int mode, bool batch, rk_plan *P,
                          std::vector<uint8_t> &blob, std::vector<InstDesc> &descs, std::vector<uint64_t> &items);
void plan_sizes(const std::vector<uint8_t> &blob, const std::vector<InstDesc> &descs, const std::vector<uint64_t> &items,
                uint64_t *blob_bytes, uint64_t *desc_bytes, uint64_t *item_bytes);
void prepare_scan_kernels();
// HIP events around one launch on s when profiling is on (kind: the
// rk_ctx_profile kernel class); slot -1 when off
hipError_t prof_begin(rk_ctx *ctx, hipStream_t s, int kind, int *slot);
hipError_t prof_end(rk_ctx *ctx, hipStream_t s, int slot);
hipError_t launch_stream_read(const void *data, uint64_t n, uint32_t *out, uint32_t grid, hipStream_t s);

// Launchers of the scan kernels of one family (kFamScreen1 / kFamScreen /
// kFamExact) and one geometry CFG of kTileCfgs.  The kernels are defined in
// rk_scan.h and instantiated in the rk_scan_*.hip translation units (split by
// family, geometry and kernel so that they compile in parallel); every other
// unit sees these declarations only.
template <int FAM, int CFG>
struct ScanGeom {
  // the general scan kernel
  static hipError_t launch(const ScanParams &p, uint32_t grid, uint32_t lds_bytes, hipStream_t s);
  static hipError_t occupancy(uint32_t lds_bytes, int *blocks);
  static hipError_t prepare();
  // the single-bucket kernel
  static hipError_t list(const ListParams *p, uint32_t grid, hipStream_t s, int *blocks);
  static hipError_t list_prepare();
};

// device translation unit
uint32_t scan_lds_bytes(int cfg, uint32_t img_cap);
hipError_t launch_scan(int cfg, int fam, const ScanParams &p, uint32_t grid, uint32_t lds_bytes, hipStream_t s);
hipError_t scan_occupancy(int cfg, int fam, uint32_t lds_bytes, int *blocks_per_cu);
hipError_t list_scan(int cfg, int fam, const ListParams *p, uint32_t grid, hipStream_t s, int *blocks_per_cu);
uint64_t scan_tmp_words(uint64_t n);
hipError_t launch_exclusive_scan(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *tmp, uint64_t *total_dev,
                                 hipStream_t s);
// the same scan when bsum already holds the sums of the counts' blocks of
// 2^kTileSumLog2 (bsum: ceil(n / 2^kTileSumLog2) + 1 entries, overwritten)
hipError_t launch_exclusive_scan_summed(const uint32_t *in, uint64_t n, uint64_t *out, uint64_t *bsum, hipStream_t s);
// sparse: fewer hits than tiles (a lane per tile); offsets1: a single
// pattern's offsets, written {0, total}, or null
hipError_t launch_compact(const uint32_t *counts, const uint64_t *offs, uint64_t ntiles, const uint64_t *slabs,
                          uint32_t slab_cap, uint64_t *out, bool sparse, uint64_t *offsets1, uint64_t total,
                          hipStream_t s);
uint64_t radix_blocks(uint64_t n);
hipError_t launch_radix(uint64_t *a, uint64_t *b, uint64_t n, uint32_t k, uint32_t *ghist, uint64_t *goff,
                        uint64_t *tmp, uint8_t *cs, uint64_t *offsets, uint64_t *positions, hipStream_t s);
// work bytes of the one-pass sorts' digit offsets for up to nh histogram
// entries of nd digits
uint64_t digit_cs_bytes(uint64_t nh, uint32_t nd);
// Records of one part's tiles as the count pass left them (dense hits: the
// collect sorts them without compacting them first): tile t's counts[t]
// records are its slab (slabs + (t - tile0) * S) when they fit, else those
// of the collect's rescan, at tile_off[t] of the direct buffer.  A radix
// block takes G consecutive tiles; blk0 is the part's first block.
struct TileSrc {
  const uint32_t *counts;    // per tile, the pass's numbering
  const uint64_t *tile_off;  // exclusive scan of counts
  const uint64_t *slabs;     // the part's slabs [tile][S]
  const uint64_t *direct;    // records of the rescanned tiles
  uint64_t tile0, ntiles;    // the part's tiles
  uint64_t blk0;             // global index of the part's first block
  uint32_t S, G;
};

hipError_t launch_radix_tiles(const TileSrc *parts, uint32_t nparts, uint64_t nblk, uint64_t n, uint32_t k,
                              uint32_t *ghist, uint64_t *goff, uint8_t *cs, uint64_t *offsets, uint64_t *positions,
                              hipStream_t s);
hipError_t launch_pid_offsets(const uint64_t *sorted, uint64_t n, uint32_t k, uint64_t *offsets, hipStream_t s);
hipError_t launch_strip(const uint64_t *rec, uint64_t n, uint64_t *pos, hipStream_t s);
hipError_t launch_window_hashes(const uint8_t *text, uint64_t n, uint32_t m, const uint64_t *xs, uint64_t cnt,
                                uint64_t *out, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint64_t words, uint32_t v, hipStream_t s);
rk_status tune_run(rk_ctx *ctx, uint64_t n, const uint32_t *lengths, uint32_t nl, const char *path);
// patterns of an instance per m-bucket (the m-class of each group's stream
// length) under a mode; npat[c] = 0 for an empty bucket
void instance_buckets(const uint8_t *bytes, const uint64_t *offs, uint32_t k, int mode, uint32_t npat[kNumMClass]);
rk_status tune_load(rk_ctx *ctx, const char *path);
rk_status static_scratch_setup(rk_ctx *ctx);

}  // namespace rk
