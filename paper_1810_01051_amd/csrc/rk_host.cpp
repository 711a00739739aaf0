// Host runtime of librk: contexts, pattern preprocessing (plans), scratch
// layout, launch orchestration of the count and collect passes, profiling and
// the scan-geometry autotuner.  Every entry point of include/rk.h except the
// server lives here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/rk.h"
#include "rk_internal.h"
#include "rk_runtime.h"

namespace rk {

// ------------------------------------------------------------ host arithmetic
// The library's own mod 2^61-1 arithmetic for d = 256 (pattern hashes are
// computed once on the host, Sec. 3.1).  256*s is a rotation of the 61-bit word.
static inline uint64_t h_mul256(uint64_t s) { return ((s << 8) & kQ) + (s >> 53); }
static inline uint64_t h_canon(uint64_t s) {
  uint64_t f = (s & kQ) + (s >> 61);
  return f >= kQ ? f - kQ : f;
}
uint64_t host_hash(const uint8_t *p, uint64_t m) {
  uint64_t s = 0;
  for (uint64_t i = 0; i < m; ++i) s = h_canon(h_mul256(s) + p[i]);
  return s;
}
// screen shift for a pattern length: the smallest power of two s with s*m >= 32
// and s >= 2 (s = 1 is the paper's shift-and-add form; s = 2 keeps the warm-up
// at 15 bytes while every byte of a window of length >= 16 still contributes)
uint32_t screen_shift(uint32_t m) {
  if (m < 8) return 8;
  if (m < 16) return 4;
  return 2;
}
uint32_t screen_hash(const uint8_t *p, uint32_t m) {
  const uint32_t s = screen_shift(m);
  uint32_t h = 0;
  for (uint32_t i = 0; i < m; ++i) h = (h << s) + p[i];
  if (s == 8 && m < 4) h &= (1u << (8 * m)) - 1u;
  return h;
}

// ------------------------------------------------------------------ errors
rk_status set_err(rk_ctx *ctx, rk_status st, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return st;
}

rk_status hip_err(rk_ctx *ctx, hipError_t e, const char *what) {
  return set_err(ctx, RK_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr, what)                 \
  do {                                           \
    hipError_t e_ = (expr);                      \
    if (e_ != hipSuccess) return hip_err(ctx, e_, what); \
  } while (0)

static inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }
static inline uint32_t next_pow2(uint32_t v) {
  uint32_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

// ------------------------------------------------------------ image building
// An instance image holds, per group of patterns, the structures the scan
// probes for every window (up to 4 register targets or a fingerprint table)
// and those it walks for candidates only (a key -> entry-run hash table, the
// entries and the pattern bytes).
//
// Screen mode groups patterns by the part of the window their shift-add hash
// covers: s=8 hashes the last 4 bytes, s=4 the last 8, s=2 the last 16, and
// bytes older than that have shifted out of the 32-bit word.  So every pattern
// of length >= 16 shares one hash stream (its key is the shift-add hash of
// its last 16 bytes), likewise 8..15 and 4..7; lengths 1..3 get one group each
// (the hash is masked to the window).  Exact mode groups by length class, each
// class keyed on the exact hash of the last l bytes, l its shortest length.
struct PatRef {
  uint32_t pid;
  const uint8_t *p;
  uint32_t m;
  uint64_t key;  // screen hash (screen groups) or exact hash (exact groups)
  uint64_t hx;   // exact hash
};

struct GroupIn {
  bool screen;
  uint32_t shift, mask;  // screen groups
  uint32_t m;            // exact groups: the length; screen groups: the shortest length
  std::vector<PatRef> pats;
};

static uint32_t screen_mask(uint32_t m) { return (screen_shift(m) == 8 && m < 4) ? (1u << (8 * m)) - 1u : 0xFFFFFFFFu; }

// group id for a pattern length under a mode.  Lengths 1..3 get one group
// each.  Screen mode: one group per shift (the span its hash covers).  Exact
// mode: one group per length class (4..7, 8..15, 16..31, 32 and longer), whose
// rolling stream hashes the last l bytes of each window, l the shortest
// pattern length of the class (at most kStreamM): every pattern of the class
// is keyed by the exact hash of its last l bytes, so a set of many lengths
// costs one stream per class instead of one per length, and a class holding
// one length hashes whole windows.
static uint32_t group_id(int mode, uint32_t m) {
  if (m < 4) return m;
  if (mode == RK_MODE_EXACT) return 200 + (uint32_t)m_class(m);
  return 100 + screen_shift(m);
}

// Cuckoo table of 32-bit keys for the per-window set test: a key sits in one
// of its two slots (ck_slot1 / ck_slot2, which the kernel computes the same
// way), so a window costs two LDS reads and two full 32-bit compares and has
// no false positives beyond hash equality.  Empty slots hold a value that is
// no key.  At most 45% of the slots are used.
static bool build_cuckoo(const std::vector<uint32_t> &keys, uint32_t bits, std::vector<uint32_t> &tab) {
  const uint32_t S = 1u << bits, sh = 32 - bits;
  std::vector<uint32_t> sorted(keys);
  std::sort(sorted.begin(), sorted.end());
  uint32_t filler = 0;
  for (uint32_t k : sorted) {
    if (k == filler) ++filler;
    else if (k > filler) break;
  }
  tab.assign(S, filler);
  std::vector<uint8_t> used(S, 0);
  uint32_t rng = 0x2545F491u;
  for (uint32_t key : keys) {
    uint32_t cur = key;
    bool placed = false;
    for (int kick = 0; kick < 1000 && !placed; ++kick) {
      const uint32_t a = ck_slot1(cur, sh), b = ck_slot2(cur, sh);
      if (!used[a]) {
        tab[a] = cur;
        used[a] = 1;
        placed = true;
      } else if (!used[b]) {
        tab[b] = cur;
        used[b] = 1;
        placed = true;
      } else {
        rng = rng * 1103515245u + 12345u;
        const uint32_t v = ((rng >> 16) & 1u) ? a : b;
        std::swap(cur, tab[v]);  // the evicted key tries its other slot next
      }
    }
    if (!placed) return false;
  }
  return true;
}

// A group serialised in two parts: what the kernel probes for every window
// (the cuckoo table, staged in LDS) and what it walks for candidates only
// (key table, entries, pattern bytes; read from the plan in device memory).
// Offsets in the descriptor are relative to the start of each part.
struct GroupBody {
  std::vector<uint8_t> lds, glob;
  BucketDesc D;
  std::vector<uint32_t> tab;  // the cuckoo table (table kinds)
};

static uint32_t put_bytes(std::vector<uint8_t> &body, const void *p, size_t bytes) {
  const uint32_t off = (uint32_t)align_up(body.size(), 16);
  body.resize(off + align_up(bytes, 16), 0);
  if (bytes) memcpy(body.data() + off, p, bytes);
  return off;
}

// Record of the entries [i, j) sharing one key: one entry inline; a run of
// one pattern under several ids (identical bytes: one comparison, then a hit
// per id) as such when it fits that encoding; else a plain run.
static uint64_t key_record(const std::vector<Entry> &ents, size_t i, size_t j) {
  if (j - i == 1) return slot_inline(ents[i].pid, ents[i].off_m);
  bool same = j - i <= kSameMaxCount && i < kSameMaxFirst;
  for (size_t q = i + 1; q < j && same; ++q) same = ents[q].off_m == ents[i].off_m;
  if (same) return slot_same((uint32_t)i, (uint32_t)(j - i), ents[i].off_m);
  return slot_run((uint32_t)i, (uint32_t)(j - i));
}

// Serialises one group.  Returns false if its keys do not fit a cuckoo table
// of at most 2^kMaxTableBits slots or it has more entries than a run can
// address (the caller then splits the group).
static bool emit_group(const GroupIn &G, GroupBody &out) {
  std::vector<PatRef> P = G.pats;
  // entries sharing the low key word (the table key) side by side
  std::stable_sort(P.begin(), P.end(), [](const PatRef &a, const PatRef &b) {
    if ((uint32_t)a.key != (uint32_t)b.key) return (uint32_t)a.key < (uint32_t)b.key;
    if (a.key != b.key) return a.key < b.key;
    if (a.m != b.m) return a.m < b.m;
    const int c = memcmp(a.p, b.p, a.m);  // identical patterns side by side
    if (c) return c < 0;
    return a.pid < b.pid;
  });
  if (P.size() > 0xFFFFu) return false;
  BucketDesc &D = out.D;
  memset(&D, 0, sizeof D);
  D.m = G.m;
  D.npat = (uint32_t)P.size();
  D.mask = G.screen ? G.mask : 0xFFFFFFFFu;
  std::vector<uint64_t> dist;
  for (const PatRef &r : P)
    if (dist.empty() || dist.back() != r.key) dist.push_back(r.key);
  std::vector<uint32_t> tkeys;
  if (!G.screen) {
    std::vector<uint32_t> lazy;
    for (uint64_t H : dist) {
      lazy.push_back((uint32_t)H);
      lazy.push_back((uint32_t)(H + kQ));
      if (H + 2 * kQ < (1ull << 62) + (1ull << 11)) lazy.push_back((uint32_t)(H + 2 * kQ));
    }
    if (lazy.size() <= 4) {
      D.kind = kListExact;
      for (int j = 0; j < 4; ++j) D.tgt[j] = lazy[j < (int)lazy.size() ? j : 0];
      D.shift = (uint32_t)(lazy.size() <= 2 ? 2u : 4u) << 8;  // compare count the kernel unrolls
    } else {
      D.kind = kTableExact;
      for (uint64_t H : dist) tkeys.push_back((uint32_t)H);  // low word of the canonical hash
    }
  } else {
    D.shift = G.shift;
    if (dist.size() <= 4) {
      D.kind = kListScreen;
      for (int j = 0; j < 4; ++j) D.tgt[j] = (uint32_t)dist[j < (int)dist.size() ? j : 0];
      D.shift |= (dist.size() == 1 ? 1u : 4u) << 8;  // compare count the kernel unrolls
    } else {
      D.kind = kTableScreen;
      for (uint64_t h : dist) tkeys.push_back((uint32_t)h);
    }
  }
  if (D.kind == kTableScreen || D.kind == kTableExact) {
    std::sort(tkeys.begin(), tkeys.end());
    tkeys.erase(std::unique(tkeys.begin(), tkeys.end()), tkeys.end());
    uint32_t bits = 6;
    while ((1u << bits) * 9u < tkeys.size() * 20u) ++bits;  // load <= 45%
    std::vector<uint32_t> tab;
    bool ok = false;
    for (; bits <= kMaxTableBits; ++bits)
      if ((ok = build_cuckoo(tkeys, bits, tab))) break;
    if (!ok) return false;
    D.fp_mask = 32 - bits;  // the kernel's slot shift
    D.fp_off = put_bytes(out.lds, tab.data(), tab.size() * 4);
    out.tab = std::move(tab);
  }
  const bool table = D.kind == kTableScreen || D.kind == kTableExact;
  std::vector<Entry> ents(P.size());
  std::vector<uint8_t> pb;
  // pattern bytes, each at a 4-byte aligned offset (the kernel compares
  // dwords); identical patterns under several ids are stored once
  uint32_t max_m = 0;
  std::unordered_map<std::string, uint32_t> stored;
  for (size_t i = 0; i < P.size(); ++i) {
    ents[i].hx = P[i].hx;
    ents[i].pid = P[i].pid;
    std::string s((const char *)P[i].p, P[i].m);
    auto it = stored.find(s);
    uint32_t off;
    if (it != stored.end()) {
      off = it->second;
    } else {
      off = (uint32_t)pb.size();
      stored.emplace(std::move(s), off);
      pb.insert(pb.end(), P[i].p, P[i].p + P[i].m);
      pb.resize(align_up(pb.size(), 4), 0);
    }
    ents[i].off_m = om_pack(off, P[i].m);  // offset relative to the pattern block
    max_m = std::max(max_m, P[i].m);
  }
  if (pb.size() > kGroupPatBytes) return false;  // split: entries address 4 MiB of pattern bytes
  pb.resize(pb.size() + 16, 0);  // the kernel reads a pattern's first 16 bytes at once, whatever its length
  if (table) {
    // one record per cuckoo slot: the run of entries whose table key sits in
    // that slot, a single entry held inline
    const uint32_t S = (uint32_t)out.tab.size(), sh = D.fp_mask;
    std::vector<uint64_t> rec(S, 0);
    for (size_t i = 0; i < P.size();) {
      size_t j = i;
      while (j < P.size() && (uint32_t)P[j].key == (uint32_t)P[i].key) ++j;
      const uint32_t h = (uint32_t)P[i].key;
      uint32_t s = ck_slot1(h, sh);
      if (out.tab[s] != h) s = ck_slot2(h, sh);
      rec[s] = key_record(ents, i, j);
      i = j;
    }
    D.ht_mask = S - 1;
    D.ht_off = put_bytes(out.glob, rec.data(), rec.size() * 8);
  } else {
    // key -> run record, open addressing
    const uint32_t S = std::max<uint32_t>(2, next_pow2(2 * (uint32_t)dist.size()));
    std::vector<uint64_t> keys(S, kEmptyKey), vals(S, 0);
    for (size_t i = 0; i < P.size();) {
      size_t j = i;
      while (j < P.size() && P[j].key == P[i].key) ++j;
      uint32_t s = ht_slot(P[i].key, S - 1);
      while (keys[s] != kEmptyKey) s = (s + 1) & (S - 1);
      keys[s] = P[i].key;
      vals[s] = key_record(ents, i, j);
      i = j;
    }
    std::vector<uint8_t> ht(S * 16);
    memcpy(ht.data(), keys.data(), S * 8);
    memcpy(ht.data() + S * 8, vals.data(), S * 8);
    D.ht_mask = S - 1;
    D.ht_off = put_bytes(out.glob, ht.data(), ht.size());
  }
  D.ent_off = put_bytes(out.glob, ents.data(), ents.size() * sizeof(Entry));
  D.pat_off = put_bytes(out.glob, pb.data(), pb.size());
  D.max_m = max_m;
  return true;
}

// Emits G, splitting its pattern list in halves while it does not fit.
static void expand_group(const GroupIn &G, std::vector<GroupBody> &bodies) {
  GroupBody gb;
  if (emit_group(G, gb) || G.pats.size() < 2) {
    bodies.push_back(std::move(gb));
    return;
  }
  GroupIn a = G, b = G;
  const size_t h = G.pats.size() / 2;
  a.pats.assign(G.pats.begin(), G.pats.begin() + h);
  b.pats.assign(G.pats.begin() + h, G.pats.end());
  expand_group(a, bodies);
  expand_group(b, bodies);
}

// Packs groups greedily into virtual instances whose LDS part (header,
// descriptors, cuckoo tables) fits kImgLimit.  Image layout:
//   [ImageHeader][BucketDesc x nb][LDS parts ...][device-memory parts ...]
static rk_status build_images(rk_ctx *ctx, const std::vector<GroupIn> &groups, uint32_t src_inst,
                              std::vector<VInst> &vinsts, std::vector<uint8_t> &blob) {
  std::vector<GroupBody> bodies;
  for (const GroupIn &G : groups) expand_group(G, bodies);
  size_t i = 0;
  while (i < bodies.size()) {
    size_t j = i;
    uint64_t lds = 0;
    while (j < bodies.size()) {
      const uint64_t hdr = sizeof(ImageHeader) + 64 * (j - i + 1);
      const uint64_t add = align_up(bodies[j].lds.size(), 16);
      if (j > i && hdr + lds + add > kImgLimit) break;
      lds += add;
      ++j;
    }
    const uint32_t hdr = (uint32_t)(sizeof(ImageHeader) + 64 * (j - i));
    if (hdr + lds > kImgLimit)
      return set_err(ctx, RK_EUNSUPPORTED, "pattern group needs %llu bytes of LDS image (limit %u)",
                     (unsigned long long)(hdr + lds), kImgLimit);
    std::vector<uint8_t> img(hdr, 0);
    std::vector<uint32_t> lds_base(j - i), glob_base(j - i);
    for (size_t b = i; b < j; ++b) {
      lds_base[b - i] = (uint32_t)img.size();
      img.insert(img.end(), bodies[b].lds.begin(), bodies[b].lds.end());
      img.resize(align_up(img.size(), 16), 0);
    }
    const uint32_t lds_bytes = (uint32_t)img.size();
    for (size_t b = i; b < j; ++b) {
      glob_base[b - i] = (uint32_t)img.size();
      img.insert(img.end(), bodies[b].glob.begin(), bodies[b].glob.end());
      img.resize(align_up(img.size(), 16), 0);
    }
    uint32_t max_m = 0, npat = 0;
    bool only_one_list = true;
    for (size_t b = i; b < j; ++b) {
      BucketDesc d = bodies[b].D;
      npat += d.npat;
      if (d.kind == kTableScreen || d.kind == kTableExact) d.fp_off += lds_base[b - i];
      d.ht_off += glob_base[b - i];
      d.ent_off += glob_base[b - i];
      d.pat_off += glob_base[b - i];
      max_m = std::max(max_m, d.max_m);
      if (d.kind != kListScreen || (d.shift >> 8) != 1u) only_one_list = false;
      memcpy(img.data() + sizeof(ImageHeader) + 64 * (b - i), &d, 64);
    }
    ImageHeader hd;
    hd.nbuckets = (uint32_t)(j - i);
    hd.bytes = (uint32_t)align_up(img.size(), 16);
    hd.max_m = max_m;
    hd.lds_bytes = lds_bytes;
    img.resize(hd.bytes, 0);
    memcpy(img.data(), &hd, sizeof hd);
    VInst v;
    v.src = src_inst;
    v.img_off = (uint32_t)align_up(blob.size(), 256);
    v.img_bytes = hd.bytes;
    v.lds_bytes = lds_bytes;
    v.nbuckets = hd.nbuckets;
    v.max_m = max_m;
    v.npat = npat;
    v.only_one_list = only_one_list;
    blob.resize(v.img_off, 0);
    blob.insert(blob.end(), img.begin(), img.end());
    vinsts.push_back(v);
    i = j;
  }
  return RK_OK;
}

static rk_status validate_patterns(rk_ctx *ctx, const uint8_t *bytes, const uint64_t *offs, uint32_t k) {
  if (k > 0 && (!offs || (!bytes && offs[k] > offs[0])))
    return set_err(ctx, RK_EINVAL, "null pattern arrays");
  if (k > RK_MAX_PID) return set_err(ctx, RK_EUNSUPPORTED, "too many patterns (%u)", k);
  for (uint32_t j = 0; j < k; ++j) {
    if (offs[j + 1] <= offs[j]) return set_err(ctx, RK_EINVAL, "pattern %u has length 0", j);
    if (offs[j + 1] - offs[j] > RK_MAX_M)
      return set_err(ctx, RK_EUNSUPPORTED, "pattern %u has length %llu > %u", j,
                     (unsigned long long)(offs[j + 1] - offs[j]), RK_MAX_M);
  }
  return RK_OK;
}

// Groups one instance's patterns (global ids from pid_base) for a mode.
static std::vector<GroupIn> group_patterns(const uint8_t *bytes, const uint64_t *offs, uint32_t k,
                                           uint32_t pid_base, int mode) {
  std::map<uint32_t, GroupIn> by;
  for (uint32_t j = 0; j < k; ++j) {
    const uint32_t m = (uint32_t)(offs[j + 1] - offs[j]);
    const uint8_t *p = bytes + offs[j];
    GroupIn &G = by[group_id(mode, m)];
    PatRef r;
    r.pid = pid_base + j;
    r.p = p;
    r.m = m;
    r.hx = host_hash(p, m);
    // the window a group's stream hashes: the shortest length of the group,
    // at most kStreamM bytes in exact mode
    const uint32_t ms = mode == RK_MODE_EXACT ? std::min(m, kStreamM) : m;
    if (G.pats.empty()) {
      G.screen = mode != RK_MODE_EXACT;
      G.shift = screen_shift(m);
      G.mask = screen_mask(m);
      G.m = ms;
    }
    G.m = std::min(G.m, ms);
    r.key = G.screen ? (uint64_t)screen_hash(p, m) : 0;
    G.pats.push_back(r);
  }
  std::vector<GroupIn> out;
  for (auto &kv : by) {
    GroupIn &G = kv.second;
    // exact keys: the exact hash of each pattern's last G.m bytes (the whole
    // pattern when it is that long)
    if (!G.screen)
      for (PatRef &r : G.pats) r.key = r.m == G.m ? r.hx : host_hash(r.p + r.m - G.m, G.m);
    out.push_back(G);
  }
  return out;
}

// Images of one instance's patterns: every group of the instance shares its
// images (one scan of the text).
rk_status build_instance_images(rk_ctx *ctx, const uint8_t *bytes, const uint64_t *offs, uint32_t k,
                                uint32_t pid_base, int mode, uint32_t src, std::vector<VInst> &vinsts,
                                std::vector<uint8_t> &blob) {
  rk_status st = validate_patterns(ctx, bytes, offs, k);
  if (st != RK_OK) return st;
  if (k == 0) return RK_OK;  // nothing to scan for
  return build_images(ctx, group_patterns(bytes, offs, k, pid_base, mode), src, vinsts, blob);
}

void instance_buckets(const uint8_t *bytes, const uint64_t *offs, uint32_t k, int mode, uint32_t npat[kNumMClass]) {
  for (int c = 0; c < kNumMClass; ++c) npat[c] = 0;
  if (k == 0) return;
  for (const GroupIn &G : group_patterns(bytes, offs, k, 0, mode)) npat[m_class(G.m)] += (uint32_t)G.pats.size();
}

}  // namespace rk

using namespace rk;

// ===================================================================== C ABI
extern "C" {

const char *rk_status_string(rk_status s) {
  switch (s) {
    case RK_OK: return "RK_OK";
    case RK_EINVAL: return "RK_EINVAL";
    case RK_ENOMEM: return "RK_ENOMEM";
    case RK_EUNSUPPORTED: return "RK_EUNSUPPORTED";
    case RK_EDEVICE: return "RK_EDEVICE";
    case RK_ENOSPACE: return "RK_ENOSPACE";
    case RK_EBUSY: return "RK_EBUSY";
    case RK_ECANCELED: return "RK_ECANCELED";
    case RK_ETIMEDOUT: return "RK_ETIMEDOUT";
  }
  return "RK_UNKNOWN";
}

rk_status rk_ctx_create(int device, uint64_t d, uint64_t q, rk_ctx **out) {
  if (!out) return RK_EINVAL;
  *out = nullptr;
  if (q != kQ || d != 256) return RK_EUNSUPPORTED;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return RK_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return RK_EDEVICE;
  rk_ctx *c = new (std::nothrow) rk_ctx();
  if (!c) return RK_ENOMEM;
  c->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete c;
    return RK_EDEVICE;
  }
  c->num_cu = prop.multiProcessorCount;
  c->arch = prop.gcnArchName;
  if (hipHostMalloc((void **)&c->pinned, 4096, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return RK_ENOMEM;
  }
  if (hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking) != hipSuccess) {
    hipHostFree(c->pinned);
    delete c;
    return RK_EDEVICE;
  }
  for (int md = 0; md < 3; ++md) {
    for (int m = 0; m <= RK_MAX_M; ++m) c->tune[md][m] = -1;
    for (int a = 0; a < kNumMClass; ++a)
      for (int b = 0; b < kNumKClass; ++b) {
        c->tune_b[md][a][b] = -1;
        for (int g = 0; g < kNumTileCfg; ++g) c->tune_bms[md][a][b][g] = -1.0;
      }
  }
  prepare_scan_kernels();
  if (static_scratch_setup(c) != RK_OK) {
    hipStreamDestroy(c->aux);
    hipHostFree(c->pinned);
    delete c;
    return RK_EDEVICE;
  }
  *out = c;
  return RK_OK;
}

void rk_ctx_destroy(rk_ctx *ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  for (auto &ev : ctx->prof_events) {
    hipEventDestroy(ev.a);
    hipEventDestroy(ev.b);
  }
  if (ctx->pinned) hipHostFree(ctx->pinned);
  if (ctx->aux) hipStreamDestroy(ctx->aux);
  delete ctx;
}

const char *rk_ctx_last_error(const rk_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

rk_status rk_ctx_set_option(rk_ctx *ctx, int option, int64_t value) {
  if (!ctx) return RK_EINVAL;
  switch (option) {
    case RK_OPT_SLAB_CAP:
      if (value < 0 || value > (1 << 20)) return set_err(ctx, RK_EINVAL, "slab cap out of range");
      ctx->slab_cap = (uint32_t)value;
      return RK_OK;
    case RK_OPT_TILE_CFG:
      if (value < -1 || value >= kNumTileCfg) return set_err(ctx, RK_EINVAL, "tile cfg out of range");
      ctx->tile_cfg = (int)value;
      return RK_OK;
    case RK_OPT_GRID:
      if (value < 0 || value > (1 << 20)) return set_err(ctx, RK_EINVAL, "grid out of range");
      ctx->grid = (uint32_t)value;
      return RK_OK;
    case RK_OPT_PROFILE:
      ctx->profile = value != 0;
      return RK_OK;
    case RK_OPT_QUEUE:
      if (value < -1 || value > 1) return set_err(ctx, RK_EINVAL, "queue option is -1, 0 or 1");
      ctx->queue = (int)value;
      return RK_OK;
  }
  return set_err(ctx, RK_EINVAL, "unknown option %d", option);
}

int rk_tile_cfg_count(void) { return kNumTileCfg; }

rk_status rk_tile_cfg(int i, uint32_t *wg, uint32_t *c, uint32_t *tile) {
  if (i < 0 || i >= kNumTileCfg) return RK_EINVAL;
  if (wg) *wg = kTileCfgs[i].wg;
  if (c) *c = kTileCfgs[i].c;
  if (tile) *tile = kTileCfgs[i].wg * kTileCfgs[i].c;
  return RK_OK;
}

rk_status rk_hash(const rk_ctx *ctx, const uint8_t *s, uint64_t m, uint64_t *out) {
  (void)ctx;
  if (!out || (m && !s)) return RK_EINVAL;
  *out = host_hash(s, m);
  return RK_OK;
}

rk_status rk_plan_create(rk_ctx *ctx, const uint8_t *bytes, const uint64_t *offs, uint32_t k, int mode,
                         rk_plan **out) {
  if (!ctx || !out) return RK_EINVAL;
  *out = nullptr;
  rk_instance inst;
  inst.text_dev = nullptr;
  inst.n = 0;
  inst.bytes_host = bytes;
  inst.offsets_host = offs;
  inst.k = k;
  return plan_build(ctx, &inst, 1, mode, false, out);
}

rk_status rk_batch_plan_create(rk_ctx *ctx, const rk_instance *inst, uint32_t count, int mode, rk_plan **out) {
  if (!ctx || !out || (count && !inst)) return RK_EINVAL;
  *out = nullptr;
  return plan_build(ctx, inst, count, mode, true, out);
}

void rk_plan_destroy(rk_plan *plan) {
  if (!plan) return;
  hipSetDevice(plan->device);
  if (plan->dev) hipFree(plan->dev);
  delete plan;
}

uint32_t rk_plan_patterns(const rk_plan *plan) { return plan ? plan->k_total : 0; }
uint64_t rk_plan_text_bytes(const rk_plan *plan) { return plan ? plan->text_bytes : 0; }

rk_status rk_scratch_size(rk_ctx *ctx, const rk_plan *plan, uint64_t n, uint64_t *bytes) {
  if (!ctx || !plan || !bytes) return RK_EINVAL;
  Layout L;
  rk_status st = make_layout(ctx, plan, n, L);
  if (st != RK_OK) return st;
  *bytes = L.total;
  return RK_OK;
}

rk_status rk_work_size(rk_ctx *ctx, const rk_plan *plan, uint64_t total, uint64_t *bytes) {
  if (!ctx || !plan || !bytes) return RK_EINVAL;
  *bytes = work_bytes_for(plan, total);
  return RK_OK;
}

rk_status rk_count(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text, uint64_t n, void *scratch,
                   uint64_t scratch_bytes, uint64_t *counts_dev, uint64_t *total_host, rk_stream s) {
  if (!ctx || !plan || !total_host) return RK_EINVAL;
  hipStream_t st = (hipStream_t)s;
  uint64_t total = 0;
  rk_status r = count_enqueue(ctx, plan, text, n, scratch, scratch_bytes, counts_dev, st);
  if (r != RK_OK) return r;
  r = count_finish(ctx, plan, scratch, st, &total);
  if (r != RK_OK) return r;
  *total_host = total;
  return RK_OK;
}

rk_status rk_collect(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text, uint64_t n, void *scratch,
                     uint64_t scratch_bytes, void *work, uint64_t work_bytes, uint64_t *offsets,
                     uint64_t *positions, uint64_t capacity, rk_stream s) {
  if (!ctx || !plan) return RK_EINVAL;
  return collect_enqueue(ctx, plan, text, n, scratch, scratch_bytes, work, work_bytes, offsets, positions,
                         capacity, (hipStream_t)s);
}

rk_status rk_window_hashes(rk_ctx *ctx, const uint8_t *text, uint64_t n, uint32_t m, const uint64_t *xs,
                           uint64_t cnt, uint64_t *out, rk_stream s) {
  if (!ctx) return RK_EINVAL;
  if (cnt == 0) return RK_OK;
  if (!text || !xs || !out) return set_err(ctx, RK_EINVAL, "null pointer");
  if (m == 0) return set_err(ctx, RK_EINVAL, "m = 0");
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  HIP_TRY(ctx, launch_window_hashes(text, n, m, xs, cnt, out, (hipStream_t)s), "window_hashes launch");
  return RK_OK;
}

rk_status rk_ctx_profile(rk_ctx *ctx, int kernel, uint64_t *launches, double *total_ms) {
  if (!ctx) return RK_EINVAL;
  HIP_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  uint64_t cnt = 0;
  double ms = 0;
  for (auto &ev : ctx->prof_events) {
    if (kernel != 3 && ev.kind != kernel) continue;
    HIP_TRY(ctx, hipEventSynchronize(ev.b), "hipEventSynchronize");
    float t = 0;
    HIP_TRY(ctx, hipEventElapsedTime(&t, ev.a, ev.b), "hipEventElapsedTime");
    ms += t;
    ++cnt;
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = ms;
  return RK_OK;
}

rk_status rk_ctx_profile_reset(rk_ctx *ctx) {
  if (!ctx) return RK_EINVAL;
  hipSetDevice(ctx->device);
  for (auto &ev : ctx->prof_events) {
    hipEventSynchronize(ev.b);
    ctx->free_events.push_back(ev);
  }
  ctx->prof_events.clear();
  return RK_OK;
}

}  // extern "C"
