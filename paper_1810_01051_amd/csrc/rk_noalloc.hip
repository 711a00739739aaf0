// A whole search (count, total, collect) that allocates nothing: its scratch
// (per-tile staging slabs, counters, tile offsets, overflow list) and its
// collect work memory (radix buffers and histograms) live in one file-scope
// device array instead of caller buffers or library allocations, for callers
// that cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid hipMalloc).
//
// The array is the same on every call on a GPU: each GPU holds one copy (its
// own address, taken once per device with hipGetSymbolAddress at context
// creation, with that device current), and it keeps the last call's contents.
// Counters are cleared by a fill kernel at the start of every count, so no
// state carries over between calls; calls that overlap on one GPU (two
// streams, two host threads) race on the array and must be serialised by the
// caller.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/rk.h"
#include "rk_internal.h"
#include "rk_runtime.h"

namespace rk {

constexpr uint64_t kStaticScratchBytes = RK_STATIC_SCRATCH_BYTES;

static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

// Device address of this device's copy of scratch, taken once per device.
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64];

rk_status static_scratch_setup(rk_ctx *ctx) {
  if (ctx->device < 0 || ctx->device >= 64) return set_err(ctx, RK_EUNSUPPORTED, "device index %d", ctx->device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_err(ctx, e != hipSuccess ? e : hipErrorInvalidSymbol, "static scratch address");
    g_scratch_ptr[ctx->device] = p;
  }
  ctx->static_scratch = g_scratch_ptr[ctx->device];
  return RK_OK;
}

}  // namespace rk

using namespace rk;

extern "C" rk_status rk_search_static(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text_dev, uint64_t n,
                                      uint64_t *offsets_dev, uint64_t *positions_dev, uint64_t capacity,
                                      uint64_t *total_host, rk_stream s) {
  if (!ctx || !plan || !total_host) return RK_EINVAL;
  *total_host = 0;
  if (!ctx->static_scratch) return set_err(ctx, RK_EDEVICE, "static scratch not set up for device %d", ctx->device);
  uint8_t *base = (uint8_t *)ctx->static_scratch;
  hipStream_t st = (hipStream_t)s;
  Layout L;
  rk_status r = make_layout(ctx, plan, n, L);
  if (r != RK_OK) return r;
  if (L.total > kStaticScratchBytes)
    return set_err(ctx, RK_ENOSPACE, "search needs %llu bytes of scratch, the static array holds %llu",
                   (unsigned long long)L.total, (unsigned long long)kStaticScratchBytes);
  r = count_enqueue(ctx, plan, text_dev, n, base, L.total, nullptr, st);
  if (r != RK_OK) return r;
  uint64_t total = 0;
  r = count_finish(ctx, plan, base, st, &total);
  if (r != RK_OK) return r;
  *total_host = total;
  const uint64_t work_off = (L.total + 255) / 256 * 256;
  const uint64_t work = work_bytes_for(plan, total);
  if (work_off + work > kStaticScratchBytes)
    return set_err(ctx, RK_ENOSPACE, "collect of %llu hits needs %llu bytes of scratch, the static array holds %llu",
                   (unsigned long long)total, (unsigned long long)(work_off + work),
                   (unsigned long long)kStaticScratchBytes);
  return collect_enqueue(ctx, plan, text_dev, n, base, L.total, work ? base + work_off : nullptr, work, offsets_dev,
                         positions_dev, capacity, st);
}

extern "C" uint64_t rk_static_scratch_bytes(void) { return kStaticScratchBytes; }
