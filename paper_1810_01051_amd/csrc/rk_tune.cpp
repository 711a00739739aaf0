// Scan-geometry autotuner.  On a synthetic DNA text it times every
// (workgroup size, windows per thread) entry of the built-in table
//   - per mode and pattern length for one pattern (the single-bucket kernel
//     of one-pattern searches), and
//   - per mode and batch bucket (m-class of the pattern lengths x class of the
//     pattern count) for the general kernel that batch work queues run,
// keeps the fastest of each (times within 2% of the best count as ties, which
// go to the lower table index: launch-to-launch spread is of that order), and
// checks that every candidate returns the same hits.  Each candidate's hits
// are recorded as a count and a digest of its offsets and positions,
// so that they can be checked against an independent search of the same text.
// The table can be saved to and loaded from a small JSON file keyed by the
// device architecture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rk.h"
#include "rk_internal.h"
#include "rk_runtime.h"

namespace rk {

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t b) { return hipMalloc(&p, b ? b : 16); }
};

// Digest of a search result: sum over the concatenation v of offsets and
// positions of v[i] * (2 i + 1), mod 2^64 (any changed, missing, extra or
// reordered entry changes it).
static uint64_t digest_of(const std::vector<uint64_t> &off, const std::vector<uint64_t> &pos) {
  uint64_t h = 0, i = 0;
  for (uint64_t v : off) h += v * (2 * i++ + 1);
  for (uint64_t v : pos) h += v * (2 * i++ + 1);
  return h;
}

struct Outcome {
  double ms = 0;
  uint64_t hits = 0, digest = 0;
};

// One candidate: a full search (count + collect) for the hit record, then
// the count pass timed with the context's launch events over several runs
// (everything on the context's own stream, readbacks included)
// (the minimum is kept; host round trips between launches do not enter).
// batch: the plan is a one-instance batch plan (general kernel, bucketed
// queue); otherwise a single-text plan.
static rk_status time_one(rk_ctx *ctx, int mode, int cfg, bool batch, const uint8_t *text, uint64_t n,
                          const std::vector<uint8_t> &bytes, const std::vector<uint64_t> &offs, Outcome *out) {
  const int saved = ctx->tile_cfg;
  ctx->tile_cfg = cfg;
  rk_plan *plan = nullptr;
  const uint32_t k = (uint32_t)offs.size() - 1;
  rk_status st;
  if (batch) {
    rk_instance I;
    I.text_dev = text;
    I.n = n;
    I.bytes_host = bytes.data();
    I.offsets_host = offs.data();
    I.k = k;
    st = rk_batch_plan_create(ctx, &I, 1, mode, &plan);
  } else {
    st = rk_plan_create(ctx, bytes.data(), offs.data(), k, mode, &plan);
  }
  ctx->tile_cfg = saved;
  if (st != RK_OK) return st;
  const uint8_t *t = batch ? nullptr : text;
  uint64_t sb = 0;
  rk_scratch_size(ctx, plan, n, &sb);
  DevBuf scratch, offd, pos, work;
  if (scratch.alloc(sb) != hipSuccess || offd.alloc((k + 1) * 8) != hipSuccess) {
    rk_plan_destroy(plan);
    return set_err(ctx, RK_ENOMEM, "autotune buffers");
  }
  uint64_t total = 0, wb = 0;
  st = rk_count(ctx, plan, t, n, scratch.p, sb, nullptr, &total, (rk_stream)ctx->aux);
  if (st == RK_OK) {
    rk_work_size(ctx, plan, total, &wb);
    if (pos.alloc(total * 8 + 8) != hipSuccess || work.alloc(wb) != hipSuccess)
      st = set_err(ctx, RK_ENOMEM, "autotune output");
  }
  if (st == RK_OK)
    st = rk_collect(ctx, plan, t, n, scratch.p, sb, work.p, wb, (uint64_t *)offd.p, (uint64_t *)pos.p, total,
                    (rk_stream)ctx->aux);
  if (st == RK_OK) {
    std::vector<uint64_t> ho(k + 1), hp(total);
    if (hipMemcpyAsync(ho.data(), offd.p, (k + 1) * 8, hipMemcpyDeviceToHost, ctx->aux) != hipSuccess ||
        (total && hipMemcpyAsync(hp.data(), pos.p, total * 8, hipMemcpyDeviceToHost, ctx->aux) != hipSuccess) ||
        hipStreamSynchronize(ctx->aux) != hipSuccess)
      st = set_err(ctx, RK_EDEVICE, "autotune readback");
    out->hits = total;
    out->digest = digest_of(ho, hp);
  }
  if (st == RK_OK) {
    const bool prof = ctx->profile;
    rk_ctx_profile_reset(ctx);
    ctx->profile = true;
    for (int rep = 0; rep < 6 && st == RK_OK; ++rep)
      st = rk_count(ctx, plan, t, n, scratch.p, sb, nullptr, &total, (rk_stream)ctx->aux);
    // several parts (geometries) cannot occur: the geometry is forced
    double best = 1e30;
    for (auto &ev : ctx->prof_events) {
      if (ev.kind != 0) continue;
      float ms = 0;
      if (hipEventSynchronize(ev.b) == hipSuccess && hipEventElapsedTime(&ms, ev.a, ev.b) == hipSuccess)
        best = std::min(best, (double)ms);
    }
    rk_ctx_profile_reset(ctx);
    ctx->profile = prof;
    out->ms = best;
  }
  rk_plan_destroy(plan);
  return st;
}

static std::string json_path_arch(const rk_ctx *ctx) {
  std::string a = ctx->arch;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

static void fill_nearest(rk_ctx *ctx, int md) {
  for (int m = 1; m <= (int)RK_MAX_M; ++m) {
    if (ctx->tune[md][m] >= 0) continue;
    for (int d = 1; d <= (int)RK_MAX_M; ++d) {
      if (m - d >= 1 && ctx->tune[md][m - d] >= 0 && ctx->tune_measured[md][m - d]) {
        ctx->tune[md][m] = ctx->tune[md][m - d];
        break;
      }
      if (m + d <= (int)RK_MAX_M && ctx->tune[md][m + d] >= 0 && ctx->tune_measured[md][m + d]) {
        ctx->tune[md][m] = ctx->tune[md][m + d];
        break;
      }
    }
  }
}

// Lengths of each m-class the bucket shapes draw from, and pattern counts of
// each k-class.
static const uint32_t kClassLo[kNumMClass] = {1, 4, 8, 16, 32};
static const uint32_t kClassHi[kNumMClass] = {3, 7, 15, 31, 64};
static const uint32_t kClassK[kNumKClass] = {1, 4, 32, 256};

// Text bytes a bucket shape is timed on: the first 1 MiB for m-class 0 (one-
// to three-byte patterns hit every few bytes), else the first 32 MiB.
static uint64_t bucket_text(uint64_t n, int mc) { return std::min<uint64_t>(n, mc == 0 ? (1u << 20) : (32u << 20)); }

// Pattern set of a bucket shape over text[0..n): k patterns, pattern j of
// length lo + j mod (hi - lo + 1), copied from the text at (n/3 + 7919 j) mod
// (n - m + 1), reversed for odd j (so that half of them rarely occur).
static void bucket_patterns(const std::vector<uint8_t> &text, uint64_t n, int mc, int kc, std::vector<uint8_t> &bytes,
                            std::vector<uint64_t> &offs) {
  const uint32_t lo = kClassLo[mc], hi = kClassHi[mc], k = kClassK[kc];
  bytes.clear();
  offs.assign(1, 0);
  for (uint32_t j = 0; j < k; ++j) {
    const uint32_t m = lo + j % (hi - lo + 1);
    const uint64_t o = (n / 3 + 7919ull * j) % (n - m + 1);
    const size_t b0 = bytes.size();
    bytes.insert(bytes.end(), text.begin() + o, text.begin() + o + m);
    if (j & 1) std::reverse(bytes.begin() + b0, bytes.end());
    offs.push_back(bytes.size());
  }
}

static int pick_best(const double *ms, int count) {
  double best = 1e30;
  for (int c = 0; c < count; ++c) best = std::min(best, ms[c]);
  int pick = 0;
  for (int c = count - 1; c >= 0; --c)
    if (ms[c] <= best * 1.02) pick = c;
  return pick;
}

rk_status tune_run(rk_ctx *ctx, uint64_t n, const uint32_t *lengths, uint32_t nl, const char *path) {
  if (!ctx || (nl && !lengths)) return RK_EINVAL;
  if (n < (1u << 16)) return set_err(ctx, RK_EINVAL, "autotune text must be at least 64 KiB");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RK_EDEVICE, "hipSetDevice failed");
  // synthetic DNA-like text from a fixed 64-bit LCG (Knuth's MMIX constants):
  // byte i = "ACGT"[x_i >> 62], x_{i+1} = 6364136223846793005 x_i + 1442695040888963407
  std::vector<uint8_t> host(n);
  uint64_t x = 0x181001051ull;
  static const uint8_t acgt[4] = {'A', 'C', 'G', 'T'};
  for (uint64_t i = 0; i < n; ++i) {
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    host[i] = acgt[x >> 62];
  }
  DevBuf text;
  if (text.alloc(n) != hipSuccess) return set_err(ctx, RK_ENOMEM, "autotune text");
  if (hipMemcpyAsync(text.p, host.data(), n, hipMemcpyHostToDevice, ctx->aux) != hipSuccess ||
      hipStreamSynchronize(ctx->aux) != hipSuccess)
    return set_err(ctx, RK_EDEVICE, "autotune upload");
  std::vector<std::string> rows, brows;
  char row[256];
  // one pattern per length: the text's bytes at n/3
  for (uint32_t li = 0; li < nl; ++li) {
    const uint32_t m = lengths[li];
    if (m == 0 || m > RK_MAX_M) return set_err(ctx, RK_EINVAL, "autotune length %u out of range", m);
    const std::vector<uint8_t> pat(host.begin() + n / 3, host.begin() + n / 3 + m);
    const std::vector<uint64_t> offs = {0, m};
    for (int mode : {RK_MODE_EXACT, RK_MODE_SCREEN}) {
      const int md = mode == RK_MODE_EXACT ? 1 : 2;
      Outcome ref, o;
      double cfg_ms[kNumTileCfg];
      for (int cfg = 0; cfg < kNumTileCfg; ++cfg) {
        rk_status st = time_one(ctx, mode, cfg, false, (const uint8_t *)text.p, n, pat, offs, &o);
        if (st != RK_OK) return st;
        if (cfg == 0) ref = o;
        else if (o.hits != ref.hits || o.digest != ref.digest)
          return set_err(ctx, RK_EDEVICE, "autotune: geometry %d disagrees with geometry 0 (m=%u)", cfg, m);
        snprintf(row, sizeof row, "{\"mode\": %d, \"m\": %u, \"cfg\": %d, \"ms\": %.6f, \"hits\": %llu, \"digest\": %llu}",
                 mode, m, cfg, o.ms, (unsigned long long)o.hits, (unsigned long long)o.digest);
        rows.push_back(row);
        cfg_ms[cfg] = o.ms;
      }
      ctx->tune[md][m] = pick_best(cfg_ms, kNumTileCfg);
      ctx->tune_measured[md][m] = 1;
    }
  }
  // batch buckets: the general kernel over a one-instance batch plan
  std::vector<uint8_t> bytes;
  std::vector<uint64_t> offs;
  for (int mode : {RK_MODE_EXACT, RK_MODE_SCREEN}) {
    const int md = mode == RK_MODE_EXACT ? 1 : 2;
    for (int mc = 0; mc < kNumMClass; ++mc)
      for (int kc = 0; kc < kNumKClass; ++kc) {
        const uint64_t nb = bucket_text(n, mc);
        bucket_patterns(host, nb, mc, kc, bytes, offs);
        Outcome ref, o;
        double cfg_ms[kNumTileCfg];
        for (int cfg = 0; cfg < kNumTileCfg; ++cfg) {
          rk_status st = time_one(ctx, mode, cfg, true, (const uint8_t *)text.p, nb, bytes, offs, &o);
          if (st != RK_OK) return st;
          if (cfg == 0) ref = o;
          else if (o.hits != ref.hits || o.digest != ref.digest)
            return set_err(ctx, RK_EDEVICE, "autotune: geometry %d disagrees with geometry 0 (bucket %d/%d)", cfg,
                           mc, kc);
          snprintf(row, sizeof row,
                   "{\"mode\": %d, \"mclass\": %d, \"kclass\": %d, \"k\": %u, \"n\": %llu, \"cfg\": %d, \"ms\": "
                   "%.6f, \"hits\": %llu, \"digest\": %llu}",
                   mode, mc, kc, kClassK[kc], (unsigned long long)nb, cfg, o.ms, (unsigned long long)o.hits,
                   (unsigned long long)o.digest);
          brows.push_back(row);
          cfg_ms[cfg] = o.ms;
          ctx->tune_bms[md][mc][kc][cfg] = o.ms * (double)(1u << 20) / (double)nb;
        }
        ctx->tune_b[md][mc][kc] = pick_best(cfg_ms, kNumTileCfg);
      }
  }
  fill_nearest(ctx, 1);
  fill_nearest(ctx, 2);
  if (path) {
    FILE *f = fopen(path, "w");
    if (!f) return set_err(ctx, RK_EINVAL, "cannot write %s", path);
    fprintf(f, "{\"arch\": \"%s\", \"n\": %llu, \"timings\": [\n", json_path_arch(ctx).c_str(),
            (unsigned long long)n);
    for (size_t i = 0; i < rows.size(); ++i) fprintf(f, "  %s%s\n", rows[i].c_str(), i + 1 < rows.size() ? "," : "");
    fprintf(f, "], \"bucket_timings\": [\n");
    for (size_t i = 0; i < brows.size(); ++i)
      fprintf(f, "  %s%s\n", brows[i].c_str(), i + 1 < brows.size() ? "," : "");
    fprintf(f, "], \"buckets\": [\n");
    bool first = true;
    for (int md = 1; md <= 2; ++md)
      for (int mc = 0; mc < kNumMClass; ++mc)
        for (int kc = 0; kc < kNumKClass; ++kc) {
          fprintf(f, "%s  {\"bmode\": %d, \"mclass\": %d, \"kclass\": %d, \"cfg\": %d}", first ? "" : ",\n", md, mc,
                  kc, ctx->tune_b[md][mc][kc]);
          first = false;
        }
    fprintf(f, "\n], \"choice\": [\n");
    first = true;
    for (int md = 1; md <= 2; ++md)
      for (int m = 1; m <= (int)RK_MAX_M; ++m)
        if (ctx->tune_measured[md][m]) {
          fprintf(f, "%s  {\"mode\": %d, \"m\": %d, \"cfg\": %d}", first ? "" : ",\n", md, m, ctx->tune[md][m]);
          first = false;
        }
    fprintf(f, "\n]}\n");
    fclose(f);
  }
  return RK_OK;
}

// Minimal reader for the file written above: the arch string, the bucket
// timings (time per MiB of each geometry for each bucket shape), the
// {"bmode": a, "mclass": b, "kclass": c, "cfg": d} objects after "buckets" and
// the {"mode": a, "m": b, "cfg": c} objects after "choice".
rk_status tune_load(rk_ctx *ctx, const char *path) {
  FILE *f = fopen(path, "r");
  if (!f) return set_err(ctx, RK_EINVAL, "cannot read %s", path);
  std::string s;
  char buf[4096];
  size_t r;
  while ((r = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, r);
  fclose(f);
  const size_t ap = s.find("\"arch\": \"");
  if (ap == std::string::npos) return set_err(ctx, RK_EINVAL, "%s: no arch", path);
  const size_t ae = s.find('"', ap + 9);
  if (s.substr(ap + 9, ae - ap - 9) != json_path_arch(ctx)) return RK_OK;  // another architecture: ignored
  size_t p = s.find("\"buckets\"");
  int md, m, cfg, mc, kc;
  if (p != std::string::npos) {
    while ((p = s.find("{\"bmode\": ", p)) != std::string::npos) {
      if (sscanf(s.c_str() + p, "{\"bmode\": %d, \"mclass\": %d, \"kclass\": %d, \"cfg\": %d}", &md, &mc, &kc, &cfg) ==
              4 &&
          md >= 1 && md <= 2 && mc >= 0 && mc < kNumMClass && kc >= 0 && kc < kNumKClass && cfg >= 0 &&
          cfg < kNumTileCfg)
        ctx->tune_b[md][mc][kc] = cfg;
      ++p;
    }
  }
  p = s.find("\"bucket_timings\"");
  if (p != std::string::npos) {
    const size_t stop = s.find("\"buckets\"", p);
    unsigned kk;
    unsigned long long nb;
    double ms;
    while ((p = s.find("{\"mode\": ", p)) != std::string::npos && p < stop) {
      if (sscanf(s.c_str() + p, "{\"mode\": %d, \"mclass\": %d, \"kclass\": %d, \"k\": %u, \"n\": %llu, \"cfg\": %d, \"ms\": %lf",
                 &md, &mc, &kc, &kk, &nb, &cfg, &ms) == 7 &&
          md >= 1 && md <= 2 && mc >= 0 && mc < kNumMClass && kc >= 0 && kc < kNumKClass && cfg >= 0 &&
          cfg < kNumTileCfg && nb > 0 && ms > 0)
        ctx->tune_bms[md][mc][kc][cfg] = ms * (double)(1u << 20) / (double)nb;
      ++p;
    }
  }
  p = s.find("\"choice\"");
  if (p == std::string::npos) return set_err(ctx, RK_EINVAL, "%s: no choice table", path);
  while ((p = s.find("{\"mode\": ", p)) != std::string::npos) {
    if (sscanf(s.c_str() + p, "{\"mode\": %d, \"m\": %d, \"cfg\": %d}", &md, &m, &cfg) == 3 && md >= 1 && md <= 2 &&
        m >= 1 && m <= (int)RK_MAX_M && cfg >= 0 && cfg < kNumTileCfg) {
      ctx->tune[md][m] = cfg;
      ctx->tune_measured[md][m] = 1;
    }
    ++p;
  }
  fill_nearest(ctx, 1);
  fill_nearest(ctx, 2);
  return RK_OK;
}

}  // namespace rk

using namespace rk;

extern "C" rk_status rk_autotune_load(rk_ctx *ctx, const char *path) {
  if (!ctx || !path) return RK_EINVAL;
  return tune_load(ctx, path);
}

extern "C" int rk_autotune_choice(const rk_ctx *ctx, int mode, uint32_t m) {
  if (!ctx || m == 0 || m > RK_MAX_M) return -1;
  if (ctx->tile_cfg >= 0) return ctx->tile_cfg;
  const int md = mode == RK_MODE_EXACT ? 1 : 2;
  return ctx->tune[md][m] >= 0 ? ctx->tune[md][m] : 0;
}

extern "C" int rk_autotune_bucket_choice(const rk_ctx *ctx, int mode, int mclass, int kclass) {
  if (!ctx || mclass < 0 || mclass >= kNumMClass || kclass < 0 || kclass >= kNumKClass) return -1;
  if (ctx->tile_cfg >= 0) return ctx->tile_cfg;
  const int md = mode == RK_MODE_EXACT ? 1 : 2;
  return ctx->tune_b[md][mclass][kclass];
}
