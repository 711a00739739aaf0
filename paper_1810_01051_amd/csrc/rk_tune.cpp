// Scan-geometry autotuner: times every (workgroup size, windows per thread)
// entry of the built-in table per mode and pattern length on a synthetic text,
// checks that every candidate returns the same hits, and keeps the fastest.
// Times within 2% of the best count as ties, which go to the lower table
// index (launch-to-launch spread is of that order).  The table can be saved to and loaded from
// a small JSON file keyed by the device architecture.
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
    if (p) hipFree(p);
  }
  hipError_t alloc(size_t b) { return hipMalloc(&p, b ? b : 16); }
};

// One candidate geometry: a full search (count + collect) for the hit
// cross-check, then the scan kernel alone timed with the context's launch
// events over several counts (the minimum is kept; host round trips between
// launches do not enter).
static rk_status time_one(rk_ctx *ctx, int mode, int cfg, const uint8_t *text, uint64_t n,
                          const std::vector<uint8_t> &pat, double *ms, std::vector<uint64_t> *hits) {
  const int saved = ctx->tile_cfg;
  ctx->tile_cfg = cfg;
  rk_plan *plan = nullptr;
  uint64_t offs[2] = {0, pat.size()};
  rk_status st = rk_plan_create(ctx, pat.data(), offs, 1, mode, &plan);
  ctx->tile_cfg = saved;
  if (st != RK_OK) return st;
  uint64_t sb = 0;
  rk_scratch_size(ctx, plan, n, &sb);
  DevBuf scratch, offd, pos;
  if (scratch.alloc(sb) != hipSuccess || offd.alloc(16) != hipSuccess) {
    rk_plan_destroy(plan);
    return set_err(ctx, RK_ENOMEM, "autotune buffers");
  }
  uint64_t total = 0;
  st = rk_count(ctx, plan, text, n, scratch.p, sb, nullptr, &total, nullptr);
  if (st == RK_OK && pos.alloc(total * 8 + 8) != hipSuccess) st = set_err(ctx, RK_ENOMEM, "autotune output");
  if (st == RK_OK)
    st = rk_collect(ctx, plan, text, n, scratch.p, sb, nullptr, 0, (uint64_t *)offd.p, (uint64_t *)pos.p, total,
                    nullptr);
  if (st == RK_OK) {
    hits->resize(total);
    if (total && hipMemcpy(hits->data(), pos.p, total * 8, hipMemcpyDeviceToHost) != hipSuccess)
      st = set_err(ctx, RK_EDEVICE, "autotune readback");
  }
  if (st == RK_OK) {
    const bool prof = ctx->profile;
    rk_ctx_profile_reset(ctx);
    ctx->profile = true;
    for (int rep = 0; rep < 6 && st == RK_OK; ++rep) st = rk_count(ctx, plan, text, n, scratch.p, sb, nullptr, &total, nullptr);
    double best = 1e30;
    for (auto &ev : ctx->prof_events) {
      if (ev.kind != 0) continue;
      float t = 0;
      if (hipEventSynchronize(ev.b) == hipSuccess && hipEventElapsedTime(&t, ev.a, ev.b) == hipSuccess)
        best = std::min(best, (double)t);
    }
    rk_ctx_profile_reset(ctx);
    ctx->profile = prof;
    *ms = best;
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

rk_status tune_run(rk_ctx *ctx, uint64_t n, const uint32_t *lengths, uint32_t nl, const char *path) {
  if (!ctx || (nl && !lengths)) return RK_EINVAL;
  if (n < 1024) return set_err(ctx, RK_EINVAL, "autotune text must be at least 1 KiB");
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RK_EDEVICE, "hipSetDevice failed");
  // synthetic DNA-like text from a fixed 64-bit LCG (Knuth's MMIX constants)
  std::vector<uint8_t> host(n);
  uint64_t x = 0x181001051ull;
  static const uint8_t acgt[4] = {'A', 'C', 'G', 'T'};
  for (uint64_t i = 0; i < n; ++i) {
    x = x * 6364136223846793005ull + 1442695040888963407ull;
    host[i] = acgt[x >> 62];
  }
  DevBuf text;
  if (text.alloc(n) != hipSuccess) return set_err(ctx, RK_ENOMEM, "autotune text");
  if (hipMemcpy(text.p, host.data(), n, hipMemcpyHostToDevice) != hipSuccess)
    return set_err(ctx, RK_EDEVICE, "autotune upload");
  std::vector<std::string> rows;
  for (uint32_t li = 0; li < nl; ++li) {
    const uint32_t m = lengths[li];
    if (m == 0 || m > RK_MAX_M) return set_err(ctx, RK_EINVAL, "autotune length %u out of range", m);
    const std::vector<uint8_t> pat(host.begin() + n / 3, host.begin() + n / 3 + m);
    for (int mode : {RK_MODE_EXACT, RK_MODE_SCREEN}) {
      const int md = mode == RK_MODE_EXACT ? 1 : 2;
      std::vector<uint64_t> ref;
      int best = -1;
      double best_ms = 1e30, cfg_ms[kNumTileCfg];
      for (int cfg = 0; cfg < kNumTileCfg; ++cfg) {
        double ms = 0;
        std::vector<uint64_t> hits;
        rk_status st = time_one(ctx, mode, cfg, (const uint8_t *)text.p, n, pat, &ms, &hits);
        if (st != RK_OK) return st;
        if (cfg == 0) ref = hits;
        else if (hits != ref)
          return set_err(ctx, RK_EDEVICE, "autotune: geometry %d disagrees with geometry 0 (m=%u)", cfg, m);
        char row[160];
        snprintf(row, sizeof row, "{\"mode\": %d, \"m\": %u, \"cfg\": %d, \"ms\": %.6f}", mode, m, cfg, ms);
        rows.push_back(row);
        cfg_ms[cfg] = ms;
        best_ms = std::min(best_ms, ms);
      }
      for (int cfg = kNumTileCfg - 1; cfg >= 0; --cfg)
        if (cfg_ms[cfg] <= best_ms * 1.02) best = cfg;
      ctx->tune[md][m] = best;
      ctx->tune_measured[md][m] = 1;
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
    fprintf(f, "], \"choice\": [\n");
    bool first = true;
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

// Minimal reader for the file written above: the arch string and the
// {"mode": a, "m": b, "cfg": c} objects after the "choice" key.
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
  size_t p = s.find("\"choice\"");
  if (p == std::string::npos) return set_err(ctx, RK_EINVAL, "%s: no choice table", path);
  int md, m, cfg;
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
