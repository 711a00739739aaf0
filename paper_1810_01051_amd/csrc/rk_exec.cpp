// Plan construction, scratch layout and the launch sequences of the count and
// collect passes (single search and batch), plus the hash dump.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/rk.h"
#include "rk_internal.h"
#include "rk_runtime.h"

namespace rk {

// images are built per real instance (defined in rk_host.cpp)
rk_status build_instance_images(rk_ctx *ctx, const uint8_t *bytes, const uint64_t *offs, uint32_t k,
                                uint32_t pid_base, int mode, uint32_t src, std::vector<VInst> &vinsts,
                                std::vector<uint8_t> &blob);

static inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

static int pick_cfg(const rk_ctx *ctx, int mode, uint32_t m) {
  if (ctx->tile_cfg >= 0) return ctx->tile_cfg;
  const int md = mode == RK_MODE_EXACT ? 1 : 2;
  if (m >= 1 && m <= RK_MAX_M && ctx->tune[md][m] >= 0) return ctx->tune[md][m];
  return 0;
}

// Scan geometry of a batch instance: the one with the least tuned time per
// MiB summed over the instance's m-buckets (each bucket timed alone by the
// autotuner; the instance's buckets share one scan of its text), else the
// tuned choice of its largest bucket, else the per-length choice.
static int instance_cfg(const rk_ctx *ctx, int mode, const uint32_t npat[kNumMClass], uint32_t max_m) {
  if (ctx->tile_cfg >= 0) return ctx->tile_cfg;
  const int md = mode == RK_MODE_EXACT ? 1 : 2;
  int best = -1;
  double best_ms = 0;
  for (int g = 0; g < kNumTileCfg; ++g) {
    double sum = 0;
    bool known = true;
    for (int c = 0; c < kNumMClass && known; ++c) {
      if (!npat[c]) continue;
      const double t = ctx->tune_bms[md][c][k_class(npat[c])][g];
      known = t >= 0;
      sum += t;
    }
    if (known && (best < 0 || sum < best_ms)) {
      best = g;
      best_ms = sum;
    }
  }
  if (best >= 0) return best;
  int cmax = 0;
  for (int c = 1; c < kNumMClass; ++c)
    if (npat[c] > npat[cmax]) cmax = c;
  if (npat[cmax] && ctx->tune_b[md][cmax][k_class(npat[cmax])] >= 0) return ctx->tune_b[md][cmax][k_class(npat[cmax])];
  return pick_cfg(ctx, mode, std::min(std::max(max_m, 1u), kStreamM));
}

static int part_family(int mode, const std::vector<VInst> &vs, const std::vector<uint32_t> &members) {
  if (mode == RK_MODE_EXACT) return kFamExact;
  for (uint32_t i : members)
    if (!vs[i].only_one_list) return kFamScreen;
  return kFamScreen1;
}

// Host half of a plan: images, and for batches the instance descriptors and
// the work-queue order.  P receives everything but device memory; the three
// byte arrays are what plan_upload copies to the device.
rk_status plan_build_host(rk_ctx *ctx, const rk_instance *inst, uint32_t count, int mode, bool batch, rk_plan *P,
                          std::vector<uint8_t> &blob, std::vector<InstDesc> &descs, std::vector<uint64_t> &items) {
  if (mode == RK_MODE_AUTO) mode = RK_MODE_SCREEN;
  if (mode != RK_MODE_EXACT && mode != RK_MODE_SCREEN) return set_err(ctx, RK_EINVAL, "unknown mode %d", mode);
  P->device = ctx->device;
  P->mode = mode;
  P->batch = batch;
  blob.clear();
  descs.clear();
  items.clear();
  uint64_t ktot = 0;
  // weight of each length (bytes x patterns) to pick one scan geometry
  std::map<uint32_t, double> mweight;
  for (uint32_t i = 0; i < count; ++i) {
    const rk_instance &I = inst[i];
    if (batch) {
      if (I.n && !I.text_dev) return set_err(ctx, RK_EINVAL, "instance %u: null text", i);
      if (((uintptr_t)I.text_dev & 15u) != 0) return set_err(ctx, RK_EINVAL, "instance %u: text not 16-byte aligned", i);
      if (I.n > RK_MAX_N) return set_err(ctx, RK_EUNSUPPORTED, "instance %u: text too long", i);
    }
    if (ktot + I.k > RK_MAX_PID) return set_err(ctx, RK_EUNSUPPORTED, "more than %u patterns in one plan", RK_MAX_PID);
    RealInst R;
    R.text = I.text_dev;
    R.n = I.n;
    R.pid_base = (uint32_t)ktot;
    R.k = I.k;
    P->insts.push_back(R);
    const size_t v0 = P->vinsts.size();
    rk_status st = build_instance_images(ctx, I.bytes_host, I.offsets_host, I.k, (uint32_t)ktot, mode, i,
                                         P->vinsts, blob);
    if (st != RK_OK) return st;
    uint32_t inst_max_m = 0;
    for (uint32_t j = 0; j < I.k; ++j) {
      const uint32_t m = (uint32_t)(I.offsets_host[j + 1] - I.offsets_host[j]);
      mweight[m] += (double)(batch ? I.n : 1) + 1.0;
      P->max_m = std::max(P->max_m, m);
      inst_max_m = std::max(inst_max_m, m);
    }
    if (batch) {
      uint32_t npat[kNumMClass];
      instance_buckets(I.bytes_host, I.offsets_host, I.k, mode, npat);
      const int g = instance_cfg(ctx, mode, npat, inst_max_m);
      for (size_t vi = v0; vi < P->vinsts.size(); ++vi) P->vinsts[vi].cfg = g;
    }
    ktot += I.k;
    P->text_bytes += batch ? I.n : 0;
  }
  P->k_total = (uint32_t)ktot;
  uint32_t best_m = 8;
  double bw = -1;
  for (auto &kv : mweight)
    if (kv.second > bw) {
      bw = kv.second;
      best_m = kv.first;
    }
  P->cfg = pick_cfg(ctx, mode, best_m);
  P->fam = mode == RK_MODE_EXACT ? kFamExact : kFamScreen1;
  for (const VInst &v : P->vinsts)
    if (mode != RK_MODE_EXACT && !v.only_one_list) P->fam = kFamScreen;
  for (const VInst &v : P->vinsts) P->img_cap = std::max(P->img_cap, v.lds_bytes);
  P->img_cap = (uint32_t)align_up(P->img_cap, 16);
  if (!batch && P->vinsts.size() == 1 && P->vinsts[0].nbuckets == 1) {
    memcpy(&P->list_desc, blob.data() + P->vinsts[0].img_off + sizeof(ImageHeader), sizeof(BucketDesc));
    P->list1 = P->list_desc.kind == kListScreen || P->list_desc.kind == kListExact;
    if (P->list1) {
      // a key table holding a single key: its record goes to the kernel directly
      const uint8_t *img = blob.data() + P->vinsts[0].img_off;
      const uint32_t S = P->list_desc.ht_mask + 1;
      const uint64_t *keys = (const uint64_t *)(img + P->list_desc.ht_off);
      uint32_t used = 0;
      uint64_t rec = 0;
      for (uint32_t s = 0; s < S; ++s)
        if (keys[s] != kEmptyKey) {
          ++used;
          rec = keys[S + s];
        }
      P->list_rec1 = used == 1 ? rec : 0;
    }
  }
  if (!batch) {
    // one text: one part, its tiles counted per search (they depend on n)
    Part pt;
    pt.cfg = P->cfg;
    pt.fam = P->fam;
    pt.img_cap = P->img_cap;
    pt.ninst = (uint32_t)P->vinsts.size();
    P->parts.assign(1, pt);
    return RK_OK;
  }
  // Batch: every instance image holds all its m-buckets (one scan of its
  // text) and takes the geometry its buckets' tuned timings favour; the
  // images of one geometry form a part, scanned by one persistent launch over
  // a work queue of (instance, tile) items, heavier images (more buckets,
  // longer patterns) first, so that a workgroup keeps one image across
  // consecutive pops.
  std::vector<uint32_t> members[kMaxParts];
  for (uint32_t vi = 0; vi < P->vinsts.size(); ++vi) members[P->vinsts[vi].cfg].push_back(vi);
  uint64_t base = 0;
  for (int c = 0; c < kNumTileCfg; ++c) {
    if (members[c].empty()) continue;
    Part pt;
    pt.cfg = c;
    pt.fam = part_family(mode, P->vinsts, members[c]);
    for (uint32_t vi : members[c]) pt.img_cap = std::max(pt.img_cap, P->vinsts[vi].lds_bytes);
    pt.img_cap = (uint32_t)align_up(pt.img_cap, 16);
    pt.inst0 = (uint32_t)descs.size();
    pt.ninst = (uint32_t)members[c].size();
    pt.tile0 = base;
    const uint32_t W = kTileCfgs[c].wg * kTileCfgs[c].c;
    std::vector<uint64_t> first(members[c].size());
    for (size_t q = 0; q < members[c].size(); ++q) {
      const VInst &v = P->vinsts[members[c][q]];
      const RealInst &R = P->insts[v.src];
      InstDesc d;
      memset(&d, 0, sizeof d);
      d.text = R.text;
      d.n = R.n;
      d.tile_base = base;
      d.ntiles = (R.n + W - 1) / W;
      d.img_off = v.img_off;
      d.lds_bytes = v.lds_bytes;
      first[q] = base;
      descs.push_back(d);
      base += d.ntiles;
    }
    pt.ntiles = base - pt.tile0;
    std::vector<uint32_t> order(members[c].size());
    for (uint32_t q = 0; q < order.size(); ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
      const VInst &x = P->vinsts[members[c][a]], &y = P->vinsts[members[c][b]];
      if (x.nbuckets != y.nbuckets) return x.nbuckets > y.nbuckets;
      return x.max_m > y.max_m;
    });
    pt.item0 = items.size();
    for (uint32_t q : order)
      for (uint64_t t = 0; t < descs[pt.inst0 + q].ntiles; ++t) items.push_back(first[q] + t);
    pt.nitems = items.size() - pt.item0;
    P->parts.push_back(pt);
  }
  P->total_tiles = base;
  P->nitems = items.size();
  if (!P->parts.empty()) {
    P->cfg = P->parts[0].cfg;
    P->fam = P->parts[0].fam;
  }
  return RK_OK;
}

// Device layout of a plan's three arrays inside one allocation.
void plan_sizes(const std::vector<uint8_t> &blob, const std::vector<InstDesc> &descs, const std::vector<uint64_t> &items,
                uint64_t *blob_bytes, uint64_t *desc_bytes, uint64_t *item_bytes) {
  *blob_bytes = align_up(std::max<size_t>(blob.size(), 16), 256);
  *desc_bytes = align_up(descs.size() * sizeof(InstDesc), 256);
  *item_bytes = align_up(items.size() * 8, 256);
}

rk_status plan_build(rk_ctx *ctx, const rk_instance *inst, uint32_t count, int mode, bool batch, rk_plan **out) {
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RK_EDEVICE, "hipSetDevice failed");
  rk_plan *P = new (std::nothrow) rk_plan();
  if (!P) return set_err(ctx, RK_ENOMEM, "plan allocation");
  std::vector<uint8_t> blob;
  std::vector<InstDesc> descs;
  std::vector<uint64_t> items;
  rk_status st = plan_build_host(ctx, inst, count, mode, batch, P, blob, descs, items);
  if (st != RK_OK) {
    delete P;
    return st;
  }
  uint64_t blob_bytes, desc_bytes, item_bytes;
  plan_sizes(blob, descs, items, &blob_bytes, &desc_bytes, &item_bytes);
  const uint64_t all = blob_bytes + desc_bytes + item_bytes;
  if (hipMalloc(&P->dev, all) != hipSuccess) {
    delete P;
    return set_err(ctx, RK_ENOMEM, "plan device memory (%llu bytes)", (unsigned long long)all);
  }
  P->blob_dev = (uint8_t *)P->dev;
  P->inst_dev = descs.empty() ? nullptr : (InstDesc *)((uint8_t *)P->dev + blob_bytes);
  P->items_dev = items.empty() ? nullptr : (uint64_t *)((uint8_t *)P->dev + blob_bytes + desc_bytes);
  // uploads on the context's own non-blocking stream: never the legacy
  // stream, which must not wait on a stream another thread is capturing
  hipError_t e = hipSuccess;
  if (!blob.empty()) e = hipMemcpyAsync(P->blob_dev, blob.data(), blob.size(), hipMemcpyHostToDevice, ctx->aux);
  if (e == hipSuccess && !descs.empty())
    e = hipMemcpyAsync(P->inst_dev, descs.data(), descs.size() * sizeof(InstDesc), hipMemcpyHostToDevice, ctx->aux);
  if (e == hipSuccess && !items.empty())
    e = hipMemcpyAsync(P->items_dev, items.data(), items.size() * 8, hipMemcpyHostToDevice, ctx->aux);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->aux);
  if (e != hipSuccess) {
    rk_status st2 = hip_err(ctx, e, "plan upload");
    hipFree(P->dev);
    delete P;
    return st2;
  }
  *out = P;
  return RK_OK;
}

rk_status make_layout(rk_ctx *ctx, const rk_plan *plan, uint64_t n, Layout &L) {
  L = Layout();
  // staging records per tile: one per 64 text bytes for a single pattern
  // (hits are rare), one per 16 for pattern sets (sampled patterns hit often);
  // a tile with more hits is rescanned by the collect pass
  auto slots = [&](uint32_t W) { return ctx->slab_cap ? ctx->slab_cap : (plan->k_total > 1 ? W / 16 : W / 64); };
  if (plan->batch) {
    for (const Part &pt : plan->parts) {
      PartRun r;
      r.tile0 = pt.tile0;
      r.ntiles = pt.ntiles;
      r.W = kTileCfgs[pt.cfg].wg * kTileCfgs[pt.cfg].c;
      r.S = slots(r.W);
      L.parts.push_back(r);
    }
    L.T = plan->total_tiles;
  } else {
    if (n > RK_MAX_N) return set_err(ctx, RK_EUNSUPPORTED, "text longer than 2^40-1 bytes");
    PartRun r;
    r.W = kTileCfgs[plan->cfg].wg * kTileCfgs[plan->cfg].c;
    L.T1 = (n + r.W - 1) / r.W;
    r.ntiles = L.T = L.T1 * plan->vinsts.size();
    r.S = slots(r.W);
    L.parts.push_back(r);
  }
  uint64_t o = 0;
  auto take = [&o](uint64_t bytes) {
    const uint64_t r = o;
    o = align_up(o + bytes, 256);
    return r;
  };
  // the counters and the tiles' block sums are one region, cleared by one
  // fill before every count pass
  L.nbsum = (L.T + (1u << kTileSumLog2) - 1) / (1u << kTileSumLog2) + 1;
  L.ctr = take(256 + L.nbsum * 8);
  L.bsum = L.ctr + 256;
  L.inst = take(plan->batch ? 0 : plan->vinsts.size() * sizeof(InstDesc));
  L.counts = take(L.T * 4);
  L.offsets = take(L.T * 8);
  L.ovf = take(L.T * 8);
  for (PartRun &r : L.parts) r.slabs = take(r.ntiles * (uint64_t)r.S * 8);
  L.total = o;
  return RK_OK;
}

struct WorkLayout {
  uint64_t nblk = 0, a = 0, b = 0, ghist = 0, goff = 0, tmp = 0, cs = 0, total = 0;
  uint64_t nh = 0;  // histogram entries the work holds
};

// work of a k-pattern collect: the compacted records (a), the ping-pong
// buffer of the 8-bit passes (b, only beyond 2,048 patterns), the digit
// histograms and their scan
static WorkLayout work_layout(uint64_t total, uint32_t k) {
  WorkLayout w;
  w.nblk = radix_blocks(total);
  uint64_t o = 0;
  auto take = [&o](uint64_t bytes) {
    const uint64_t r = o;
    o = align_up(o + bytes, 256);
    return r;
  };
  // digit histograms: 256 per 1024-record block (8-bit passes) or up to 2048
  // per 8192-record block (one pass of 9..11 bits), whichever is larger
  const uint64_t nh = std::max<uint64_t>(256 * w.nblk, 2048 * ((total + 8191) / 8192));
  w.a = take(total * 8);
  w.b = k > 2048 ? take(total * 8) : w.a;
  w.ghist = take(nh * 4);
  w.goff = take(nh * 8);
  w.tmp = take(scan_tmp_words(nh) * 8);
  w.cs = take(digit_cs_bytes(nh, 2048));
  w.total = o;
  w.nh = nh;
  return w;
}

uint64_t work_bytes_for(const rk_plan *plan, uint64_t total) {
  if (plan->k_total <= 1) return 0;
  return work_layout(total, plan->k_total).total;
}

hipError_t prof_begin(rk_ctx *ctx, hipStream_t s, int kind, int *slot) {
  *slot = -1;
  if (!ctx->profile) return hipSuccess;
  ProfEvent ev;
  if (!ctx->free_events.empty()) {
    ev = ctx->free_events.back();
    ctx->free_events.pop_back();
  } else {
    hipError_t e = hipEventCreate(&ev.a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&ev.b);
    if (e != hipSuccess) return e;
  }
  ev.kind = kind;
  ctx->prof_events.push_back(ev);
  *slot = (int)ctx->prof_events.size() - 1;
  return hipEventRecord(ev.a, s);
}

hipError_t prof_end(rk_ctx *ctx, hipStream_t s, int slot) {
  if (slot < 0) return hipSuccess;
  return hipEventRecord(ctx->prof_events[slot].b, s);
}

static uint32_t scan_grid(rk_ctx *ctx, int cfg, int fam, uint32_t lds, uint64_t nitems) {
  if (ctx->grid) return (uint32_t)std::min<uint64_t>(ctx->grid, std::max<uint64_t>(nitems, 1));
  int blocks = 0;
  if (scan_occupancy(cfg, fam, lds, &blocks) != hipSuccess || blocks < 1) blocks = 1;
  const uint64_t g = (uint64_t)ctx->num_cu * (uint64_t)blocks;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, nitems));
}

// Blocks per resident slot of the single-bucket scan's grid.
constexpr uint32_t kListGridMul = 32;

// Fills ScanParams common to the count pass and the rescan of part pi.
static void base_params(const rk_plan *plan, const Layout &L, uint32_t pi, uint8_t *sc, ScanParams &p) {
  memset(&p, 0, sizeof p);
  const Part &pt = plan->parts[pi];
  const PartRun &r = L.parts[pi];
  p.inst = plan->batch ? plan->inst_dev + pt.inst0 : (const InstDesc *)(sc + L.inst);
  p.ninst = pt.ninst;
  p.img_cap = pt.img_cap;
  p.blob = plan->blob_dev;
  p.tile_counts = (uint32_t *)(sc + L.counts);
  p.slab_cap = r.S;
  p.tile0 = r.tile0;
  p.total = (unsigned long long *)(sc + L.ctr);
  p.blk_sums = (unsigned long long *)(sc + L.bsum);
  p.ovf_count = (uint32_t *)(sc + L.ctr + kCtrOvf) + pi;
  p.ovf_list = (uint64_t *)(sc + L.ovf) + r.tile0;  // the part's own overflow list
  p.grab = 1;
}

// Instance descriptors of a single-text plan's text (one per virtual
// instance) into the scratch; nothing for batch plans, whose descriptors
// live in the plan.
static hipError_t upload_insts(const rk_plan *plan, const Layout &L, uint8_t *sc, const uint8_t *text, uint64_t n,
                               hipStream_t s) {
  if (plan->batch || plan->vinsts.empty()) return hipSuccess;
  std::vector<InstDesc> d(plan->vinsts.size());
  for (size_t i = 0; i < d.size(); ++i) {
    memset(&d[i], 0, sizeof(InstDesc));
    d[i].text = text;
    d[i].n = n;
    d[i].tile_base = L.T1 * i;
    d[i].ntiles = L.T1;
    d[i].img_off = plan->vinsts[i].img_off;
    d[i].lds_bytes = plan->vinsts[i].lds_bytes;
  }
  // hipMemcpyAsync from pageable memory stages the data before returning
  return hipMemcpyAsync(sc + L.inst, d.data(), d.size() * sizeof(InstDesc), hipMemcpyHostToDevice, s);
}

rk_status count_enqueue(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text, uint64_t n, void *scratch,
                        uint64_t scratch_bytes, uint64_t *counts, hipStream_t s) {
  if (plan->device != ctx->device) return set_err(ctx, RK_EINVAL, "plan belongs to another device");
  if (plan->batch) {
    if (text) return set_err(ctx, RK_EINVAL, "batch plans take text_dev = NULL");
  } else {
    if (n && !text) return set_err(ctx, RK_EINVAL, "null text");
    if (((uintptr_t)text & 15u) != 0) return set_err(ctx, RK_EINVAL, "text_dev must be 16-byte aligned");
  }
  Layout L;
  rk_status st = make_layout(ctx, plan, n, L);
  if (st != RK_OK) return st;
  if (scratch_bytes < L.total) return set_err(ctx, RK_ENOSPACE, "scratch needs %llu bytes, got %llu",
                                              (unsigned long long)L.total, (unsigned long long)scratch_bytes);
  if (!scratch) return set_err(ctx, RK_EINVAL, "null scratch");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RK_EDEVICE, "hipSetDevice failed");
  uint8_t *sc = (uint8_t *)scratch;
  hipError_t e;
  const bool use_queue = ctx->queue == 1 || (ctx->queue == -1 && plan->batch);
  // one text, one bucket with register targets: the single-bucket kernel,
  // which takes the text itself (the general kernel reads it through the
  // instance descriptors, uploaded here for it and by a rescan)
  const bool list = plan->list1 && !use_queue;
  if (!list) {
    e = upload_insts(plan, L, sc, text, n, s);
    if (e != hipSuccess) return hip_err(ctx, e, "instance upload");
  }
  e = launch_fill_u32((uint32_t *)(sc + L.ctr), 64 + 2 * L.nbsum, 0u, s);
  if (e != hipSuccess) return hip_err(ctx, e, "counter reset");
  if (counts) {
    e = launch_fill_u32((uint32_t *)counts, 2ull * plan->k_total, 0u, s);
    if (e != hipSuccess) return hip_err(ctx, e, "per-pattern count reset");
  }
  if (L.T == 0) return RK_OK;
  int slot;
  if (list) {
    const PartRun &r = L.parts[0];
    ListParams lp;
    memset(&lp, 0, sizeof lp);
    lp.text = text;
    lp.n = n;
    lp.ntiles = L.T;
    lp.gimg = plan->blob_dev + plan->vinsts[0].img_off;
    lp.D = plan->list_desc;
    lp.rot = (8u * plan->list_desc.m) % 61u;
    lp.slab_cap = r.S;
    lp.rec1 = plan->list_rec1;
    lp.tile_counts = (uint32_t *)(sc + L.counts);
    lp.out = (uint64_t *)(sc + r.slabs);
    lp.total = (unsigned long long *)(sc + L.ctr);
    lp.blk_sums = (unsigned long long *)(sc + L.bsum);
    lp.ovf_count = (uint32_t *)(sc + L.ctr + kCtrOvf);
    lp.ovf_list = (uint64_t *)(sc + L.ovf);
    lp.pid_counts = (unsigned long long *)counts;
    // The grid is kListGridMul times what is resident at once: blocks of a
    // few tiles each, dispatched as others finish, scan faster than one
    // persistent block per slot (config 2: 5.7 against 5.2 TB/s).
    uint32_t grid = ctx->grid;
    if (!grid) {
      int blocks = 0;
      if (list_scan(plan->cfg, plan->fam, nullptr, 0, nullptr, &blocks) != hipSuccess || blocks < 1) blocks = 1;
      grid = (uint32_t)ctx->num_cu * (uint32_t)blocks * kListGridMul;
    }
    grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(grid, L.T));
    e = prof_begin(ctx, s, 0, &slot);
    if (e != hipSuccess) return hip_err(ctx, e, "profiling event");
    e = list_scan(plan->cfg, plan->fam, &lp, grid, s, nullptr);
    if (e != hipSuccess) return hip_err(ctx, e, "scan launch");
    e = prof_end(ctx, s, slot);
    if (e != hipSuccess) return hip_err(ctx, e, "profiling event");
  } else {
    // one persistent launch per part (batches: per scan geometry)
    for (uint32_t pi = 0; pi < plan->parts.size(); ++pi) {
      const Part &pt = plan->parts[pi];
      const PartRun &r = L.parts[pi];
      if (r.ntiles == 0) continue;
      ScanParams p;
      base_params(plan, L, pi, sc, p);
      p.items = plan->batch ? plan->items_dev + pt.item0 : nullptr;
      p.nitems = plan->batch ? pt.nitems : r.ntiles;
      p.out = (uint64_t *)(sc + r.slabs);
      p.pid_counts = (unsigned long long *)counts;
      if (use_queue) p.queue = (uint32_t *)(sc + L.ctr + kCtrQueue) + pi;
      const uint32_t lds = scan_lds_bytes(pt.cfg, pt.img_cap);
      const uint32_t grid = scan_grid(ctx, pt.cfg, pt.fam, lds, p.nitems);
      e = prof_begin(ctx, s, 0, &slot);
      if (e != hipSuccess) return hip_err(ctx, e, "profiling event");
      e = launch_scan(pt.cfg, pt.fam, p, grid, lds, s);
      if (e != hipSuccess) return hip_err(ctx, e, "scan launch");
      e = prof_end(ctx, s, slot);
      if (e != hipSuccess) return hip_err(ctx, e, "profiling event");
    }
  }
  CountMemo &mm = ctx->memo[ctx->memo_next++ % 16];
  mm.scratch = scratch;
  mm.plan = plan;
  mm.n = n;
  mm.total = ~0ull;  // filled by count_finish
  mm.overflow = 0xFFFFFFFFu;
  return RK_OK;
}

rk_status count_finish(rk_ctx *ctx, const rk_plan *plan, void *scratch, hipStream_t s, uint64_t *total) {
  hipError_t e = hipMemcpyAsync(ctx->pinned, scratch, 64, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_err(ctx, e, "total readback");
  // A count pass of a few GiB takes about a millisecond, less than a blocking
  // wait adds in wake-up latency: the stream is polled for up to kSpinUs,
  // then waited for.
  constexpr int64_t kSpinUs = 4000;
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    e = hipStreamQuery(s);
    if (e != hipErrorNotReady) break;
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(kSpinUs)) {
      e = hipStreamSynchronize(s);
      break;
    }
  }
  if (e != hipSuccess) return hip_err(ctx, e, "scan");
  *total = ctx->pinned[0];
  const uint32_t ovf = ovf_total(ctx->pinned);
  for (auto &mm : ctx->memo)
    if (mm.scratch == scratch && mm.plan == plan) {
      mm.total = *total;
      mm.overflow = ovf;
    }
  return RK_OK;
}

rk_status collect_enqueue(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text, uint64_t n, void *scratch,
                          uint64_t scratch_bytes, void *work, uint64_t work_bytes, uint64_t *offsets,
                          uint64_t *positions, uint64_t capacity, hipStream_t s) {
  if (!offsets) return set_err(ctx, RK_EINVAL, "null offsets");
  Layout L;
  rk_status st = make_layout(ctx, plan, n, L);
  if (st != RK_OK) return st;
  if (scratch_bytes < L.total || !scratch) return set_err(ctx, RK_ENOSPACE, "scratch too small");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RK_EDEVICE, "hipSetDevice failed");
  uint8_t *sc = (uint8_t *)scratch;
  // total of the matching count pass
  uint64_t total = ~0ull;
  uint32_t overflow = 0xFFFFFFFFu;
  for (auto &mm : ctx->memo)
    if (mm.scratch == scratch && mm.plan == plan && mm.n == n && mm.total != ~0ull) {
      total = mm.total;
      overflow = mm.overflow;
    }
  if (total == ~0ull) {
    hipError_t e = hipMemcpyAsync(ctx->pinned, sc + L.ctr, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(ctx, e, "total readback");
    total = ctx->pinned[0];
  }
  return collect_enqueue_known(ctx, plan, text, n, scratch, scratch_bytes, work, work_bytes, offsets, positions, capacity,
                               total, overflow, s);
}

// Collect with the count pass's total and overflowed-tile count given by the
// caller (overflow = all ones: unknown, the rescan is launched).
rk_status collect_enqueue_known(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text, uint64_t n, void *scratch,
                                uint64_t scratch_bytes,
                                void *work, uint64_t work_bytes, uint64_t *offsets, uint64_t *positions,
                                uint64_t capacity, uint64_t total, uint32_t overflow, hipStream_t s) {
  Layout L;
  rk_status st = make_layout(ctx, plan, n, L);
  if (st != RK_OK) return st;
  uint8_t *sc = (uint8_t *)scratch;
  hipError_t e;
  if (capacity < total) return set_err(ctx, RK_ENOSPACE, "positions capacity %llu < %llu hits",
                                       (unsigned long long)capacity, (unsigned long long)total);
  if (total && !positions) return set_err(ctx, RK_EINVAL, "null positions");
  const uint32_t k = plan->k_total;
  const uint64_t need = work_bytes_for(plan, total);
  if (work_bytes < need || (need && !work))
    return set_err(ctx, RK_ENOSPACE, "work needs %llu bytes, got %llu", (unsigned long long)need,
                   (unsigned long long)work_bytes);
  int slot;
  e = prof_begin(ctx, s, 2, &slot);
  if (e != hipSuccess) return hip_err(ctx, e, "profiling event");
  if (k == 0) {
    e = launch_fill_u32((uint32_t *)offsets, 2, 0u, s);
    if (e != hipSuccess) return hip_err(ctx, e, "offsets");
    return hip_err_or_ok(ctx, prof_end(ctx, s, slot));
  }
  if (total == 0) {
    // every count is zero
    e = launch_fill_u32((uint32_t *)offsets, 2ull * (k + 1), 0u, s);
    if (e != hipSuccess) return hip_err(ctx, e, "offsets");
    return hip_err_or_ok(ctx, prof_end(ctx, s, slot));
  }
  uint64_t *tile_off = (uint64_t *)(sc + L.offsets);
  e = launch_exclusive_scan_summed((const uint32_t *)(sc + L.counts), L.T, tile_off, (uint64_t *)(sc + L.bsum), s);
  if (e != hipSuccess) return hip_err(ctx, e, "tile scan");
  WorkLayout WL = work_layout(total, k);
  uint64_t *target = k == 1 ? positions : (uint64_t *)((uint8_t *)work + WL.a);
  // Dense hits (at least 64 per tile on average) up to 2,048 patterns: the
  // sort reads the records from the slabs, G tiles per radix block (8,192 to
  // 32,768 records), and the compaction is skipped; the rescan below still
  // writes the overflowed tiles' records to the work buffer.
  TileSrc tsrc[kMaxParts];
  uint32_t ntsrc = 0;
  uint64_t tblk = 0;
  bool from_slabs = false;
  if (k > 1 && k <= 2048 && total >= 64 * L.T && L.parts.size() <= (size_t)kMaxParts) {
    uint32_t bits = 8;
    while ((1u << bits) < k) ++bits;
    // records per block: 32,768 once there are 1,024 such blocks (longer runs
    // per digit and block make the scatter's writes fuller lines), down to
    // 8,192 for fewer hits (blocks enough to fill the chip)
    const uint64_t rb = std::min<uint64_t>(32768, std::max<uint64_t>(8192, total / 1024));
    const uint32_t G = (uint32_t)std::max<uint64_t>(1, (rb * L.T + total - 1) / total);
    for (const PartRun &r : L.parts) {
      TileSrc &t = tsrc[ntsrc++];
      t.counts = (const uint32_t *)(sc + L.counts);
      t.tile_off = tile_off;
      t.slabs = (const uint64_t *)(sc + r.slabs);
      t.direct = target;
      t.tile0 = r.tile0;
      t.ntiles = r.ntiles;
      t.blk0 = tblk;
      t.S = r.S;
      t.G = G;
      tblk += (r.ntiles + G - 1) / G;
    }
    from_slabs = tblk > 0 && (1ull << bits) * tblk <= WL.nh;
  }
  // a single pattern's offsets ({0, total}) come from the first compaction
  uint64_t *offsets1 = k == 1 ? offsets : nullptr;
  for (const PartRun &r : L.parts) {
    if (from_slabs) break;
    if (r.ntiles == 0) continue;
    e = launch_compact((const uint32_t *)(sc + L.counts) + r.tile0, tile_off + r.tile0, r.ntiles,
                       (const uint64_t *)(sc + r.slabs), r.S, target, total < L.T, offsets1, total, s);
    if (e != hipSuccess) return hip_err(ctx, e, "compact");
    offsets1 = nullptr;
  }
  e = prof_end(ctx, s, slot);
  if (e != hipSuccess) return hip_err(ctx, e, "profiling event");
  // rescan of tiles whose hits did not fit their slab, part by part (each
  // part's count read on the device; skipped when the count pass reported none)
  if (overflow != 0) {
    // the rescan runs the general kernel, which reads the text through the
    // instance descriptors (a single-bucket count did not upload them)
    if (!plan->batch && !plan->vinsts.empty()) {
      if (!text) return set_err(ctx, RK_EINVAL, "the rescan of overflowed tiles needs text_dev");
      e = upload_insts(plan, L, sc, text, n, s);
      if (e != hipSuccess) return hip_err(ctx, e, "instance upload");
    }
    for (uint32_t pi = 0; pi < plan->parts.size(); ++pi) {
      const Part &pt = plan->parts[pi];
      const PartRun &r = L.parts[pi];
      if (r.ntiles == 0) continue;
      ScanParams p;
      base_params(plan, L, pi, sc, p);
      p.items = p.ovf_list;
      p.nitems = r.ntiles;
      p.nitems_dev = p.ovf_count;
      p.out = target;
      p.tile_offsets = tile_off;
      p.direct = 1;
      const uint32_t lds = scan_lds_bytes(pt.cfg, pt.img_cap);
      const uint32_t grid =
          std::min<uint32_t>(scan_grid(ctx, pt.cfg, pt.fam, lds, r.ntiles), (uint32_t)ctx->num_cu);
      e = prof_begin(ctx, s, 1, &slot);
      if (e != hipSuccess) return hip_err(ctx, e, "profiling event");
      e = launch_scan(pt.cfg, pt.fam, p, grid, lds, s);
      if (e != hipSuccess) return hip_err(ctx, e, "rescan launch");
      e = prof_end(ctx, s, slot);
      if (e != hipSuccess) return hip_err(ctx, e, "profiling event");
    }
  }
  if (k == 1) return RK_OK;  // offsets written by the compaction
  e = prof_begin(ctx, s, 2, &slot);
  if (e != hipSuccess) return hip_err(ctx, e, "profiling event");
  {
    uint8_t *wk = (uint8_t *)work;
    if (from_slabs)
      e = launch_radix_tiles(tsrc, ntsrc, tblk, total, k, (uint32_t *)(wk + WL.ghist), (uint64_t *)(wk + WL.goff),
                             wk + WL.cs, offsets, positions, s);
    else
      e = launch_radix((uint64_t *)(wk + WL.a), (uint64_t *)(wk + WL.b), total, k, (uint32_t *)(wk + WL.ghist),
                       (uint64_t *)(wk + WL.goff), (uint64_t *)(wk + WL.tmp), wk + WL.cs, offsets, positions, s);
    if (e != hipSuccess) return hip_err(ctx, e, "radix sort");
  }
  e = prof_end(ctx, s, slot);
  if (e != hipSuccess) return hip_err(ctx, e, "profiling event");
  return RK_OK;
}

}  // namespace rk

using namespace rk;

extern "C" rk_status rk_scan_dump(rk_ctx *ctx, const uint8_t *text, uint64_t n, uint32_t m, uint64_t stride,
                                  uint64_t *out, uint64_t cap, int kernel, rk_stream s) {
  if (!ctx) return RK_EINVAL;
  if (m == 0) return set_err(ctx, RK_EINVAL, "m = 0");
  if (m > kStreamM)
    return set_err(ctx, RK_EUNSUPPORTED, "m > %u: the scans roll windows of up to %u bytes (rk_window_hashes "
                   "evaluates any length)", kStreamM, kStreamM);
  if (stride == 0) return set_err(ctx, RK_EINVAL, "stride = 0");
  if (kernel != 0 && kernel != 1) return set_err(ctx, RK_EINVAL, "kernel is 0 (general) or 1 (single-bucket)");
  if (n < m) return RK_OK;
  if (!text || !out) return set_err(ctx, RK_EINVAL, "null pointer");
  if (((uintptr_t)text & 15u) != 0) return set_err(ctx, RK_EINVAL, "text_dev must be 16-byte aligned");
  if (n > RK_MAX_N) return set_err(ctx, RK_EUNSUPPORTED, "text too long");
  const uint64_t cnt = (n - m) / stride + 1;
  if (cap < cnt) return set_err(ctx, RK_ENOSPACE, "dump needs %llu entries", (unsigned long long)cnt);
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RK_EDEVICE, "hipSetDevice failed");
  hipStream_t st = (hipStream_t)s;
  const int cfg = pick_cfg(ctx, RK_MODE_EXACT, m);
  const uint32_t W = kTileCfgs[cfg].wg * kTileCfgs[cfg].c;
  const uint64_t ntiles = (n + W - 1) / W;
  BucketDesc d;
  memset(&d, 0, sizeof d);
  d.m = m;
  d.kind = kDump;
  d.mask = 0xFFFFFFFFu;
  hipError_t e;
  if (kernel == 1) {
    ListParams lp;
    memset(&lp, 0, sizeof lp);
    lp.text = text;
    lp.n = n;
    lp.ntiles = ntiles;
    lp.D = d;
    lp.rot = (8u * m) % 61u;
    lp.dump_out = out;
    lp.dump_stride = stride;
    lp.dump_cap = cap;
    uint32_t grid = ctx->grid;
    if (!grid) {
      int blocks = 0;
      if (list_scan(cfg, kFamExact, nullptr, 0, nullptr, &blocks) != hipSuccess || blocks < 1) blocks = 1;
      grid = (uint32_t)ctx->num_cu * (uint32_t)blocks;
    }
    grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(grid, ntiles));
    e = list_scan(cfg, kFamExact, &lp, grid, st, nullptr);
    if (e != hipSuccess) return hip_err(ctx, e, "dump launch");
    e = hipStreamSynchronize(st);
    return e == hipSuccess ? RK_OK : hip_err(ctx, e, "dump");
  }
  // image: header + one kDump bucket; then the instance descriptor
  uint8_t host[256];
  memset(host, 0, sizeof host);
  ImageHeader hd = {1u, 128u, m, 128u};
  memcpy(host, &hd, sizeof hd);
  memcpy(host + sizeof hd, &d, sizeof d);
  InstDesc I;
  memset(&I, 0, sizeof I);
  I.text = text;
  I.n = n;
  I.tile_base = 0;
  I.ntiles = ntiles;
  I.img_off = 0;
  I.lds_bytes = 128;
  memcpy(host + 128, &I, sizeof I);
  if (!ctx->dump_dev) {
    e = hipMalloc(&ctx->dump_dev, 256);
    if (e != hipSuccess) return hip_err(ctx, e, "dump buffer");
  }
  e = hipMemcpyAsync(ctx->dump_dev, host, 256, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_err(ctx, e, "dump upload");
  ScanParams p;
  memset(&p, 0, sizeof p);
  p.inst = (const InstDesc *)((uint8_t *)ctx->dump_dev + 128);
  p.ninst = 1;
  p.img_cap = 128;
  p.blob = (const uint8_t *)ctx->dump_dev;
  p.nitems = I.ntiles;
  p.direct = 1;
  p.dump_out = out;
  p.dump_stride = stride;
  p.dump_cap = cap;
  const uint32_t lds = scan_lds_bytes(cfg, 128);
  const uint32_t grid = scan_grid(ctx, cfg, kFamExact, lds, I.ntiles);
  e = launch_scan(cfg, kFamExact, p, grid, lds, st);
  if (e != hipSuccess) return hip_err(ctx, e, "dump launch");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_err(ctx, e, "dump");
  return RK_OK;
}

extern "C" rk_status rk_autotune(rk_ctx *ctx, uint64_t n, const uint32_t *lengths, uint32_t nlengths,
                                 const char *path) {
  return tune_run(ctx, n, lengths, nlengths, path);
}

extern "C" rk_status rk_stream_read(rk_ctx *ctx, const void *data, uint64_t n, uint32_t *out, uint32_t grid,
                                    rk_stream s) {
  if (!ctx) return RK_EINVAL;
  if (!data || !out || grid == 0 || (n & 15u) || ((uintptr_t)data & 15u))
    return set_err(ctx, RK_EINVAL, "stream_read: 16-byte aligned data, n a multiple of 16, grid > 0");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RK_EDEVICE, "hipSetDevice failed");
  int slot = -1;
  hipError_t e = prof_begin(ctx, (hipStream_t)s, 4, &slot);
  if (e == hipSuccess) e = launch_stream_read(data, n, out, grid, (hipStream_t)s);
  if (e == hipSuccess) e = prof_end(ctx, (hipStream_t)s, slot);
  return e == hipSuccess ? RK_OK : hip_err(ctx, e, "stream_read");
}
