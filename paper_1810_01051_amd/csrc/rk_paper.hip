// The paper's own GPU procedure (Shah & Oza, Sec. 3.1), kept as a mode of its
// own so that the paper's experiments (threads per block, pattern length) can
// be rerun on MI355X next to the tiled scans:
//   - one thread per text offset x, x = (block index) * (threads per block) +
//     thread index, the block index formed from a grid of up to three
//     dimensions as the paper does;
//   - the thread hashes the m bytes at T + x with the paper's shift-and-add
//     hash h <- (h << 1) + c, read straight from device memory (no tile, no
//     rolling), in a 32-bit word (the paper leaves the word width open; the
//     hash is the polynomial hash with d = 2, q = 2^32);
//   - if the hash equals the pattern's (computed once on the host) the m bytes
//     are compared, and the result array gets 1 at x for a match.
// Deviations: the result byte is written for every x (0 or 1), so the array
// needs no clearing; the device-side print of each match is not done.  The
// positions of the set bytes are gathered afterwards (rk_paper_positions) in
// ascending order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "../../include/rk.h"
#include "rk_dev.h"
#include "rk_internal.h"
#include "rk_runtime.h"

namespace rk {

__global__ void paper_kernel(const uint8_t *T, uint64_t nwin, const uint8_t *P, uint32_t m, uint32_t hx,
                             uint8_t *result, uint32_t *hash_out) {
  const uint64_t block = blockIdx.x + (uint64_t)blockIdx.y * gridDim.x + (uint64_t)gridDim.x * gridDim.y * blockIdx.z;
  const uint64_t x = block * blockDim.x + threadIdx.x;
  if (x < nwin) {  // x <= n - m
    uint32_t hy = 0;
    for (uint32_t i = 0; i < m; ++i) hy = (hy << 1) + T[x + i];
    bool match = hy == hx;
    if (match) {
      for (uint32_t i = 0; i < m; ++i)
        if (P[i] != T[x + i]) {
          match = false;
          break;
        }
    }
    result[x] = match ? 1 : 0;
    if (hash_out) hash_out[x] = hy;
  }
}

// ---------------------------------------------- flags -> ascending positions
constexpr uint32_t kFlagWG = 256;
constexpr uint32_t kFlagBlock = kFlagWG * 64;  // flags per block (64 per thread)

// count of set flags per block of kFlagBlock
__global__ __launch_bounds__(kFlagWG) void flag_counts(const uint8_t *flags, uint64_t nf, uint32_t *counts) {
  const uint64_t base = (uint64_t)blockIdx.x * kFlagBlock;
  uint32_t c = 0;
  for (uint32_t j = 0; j < 64; ++j) {
    const uint64_t i = base + (uint64_t)j * kFlagWG + threadIdx.x;
    if (i < nf) c += flags[i] != 0;
  }
  for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
  __shared__ uint32_t red[kFlagWG / 64];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (uint32_t w = 0; w < kFlagWG / 64; ++w) t += red[w];
    counts[blockIdx.x] = t;
  }
}

// Writes the positions of the set flags of each block, in ascending order,
// from the block's offset: the block walks its flags in rounds of kFlagWG
// consecutive flags, ranking each round with wave ballots.
__global__ __launch_bounds__(kFlagWG) void flag_positions(const uint8_t *flags, uint64_t nf, const uint64_t *offs,
                                                          uint64_t *pos) {
  __shared__ uint32_t wsum[kFlagWG / 64];
  const uint64_t base = (uint64_t)blockIdx.x * kFlagBlock;
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t o = offs[blockIdx.x];
  for (uint32_t j = 0; j < 64; ++j) {
    const uint64_t i = base + (uint64_t)j * kFlagWG + threadIdx.x;
    const bool f = i < nf && flags[i] != 0;
    const uint64_t b = ballot(f);
    __syncthreads();
    if (lane == 0) wsum[wave] = (uint32_t)__builtin_popcountll(b);
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (uint32_t w = 0; w < kFlagWG / 64; ++w) {
      before += w < wave ? wsum[w] : 0u;
      tot += wsum[w];
    }
    if (f) pos[o + before + (uint32_t)__builtin_popcountll(b & ((1ull << lane) - 1ull))] = i;
    o += tot;
  }
}

static rk_status paper_grid(rk_ctx *ctx, uint64_t nwin, uint32_t tpb, dim3 *grid) {
  const uint64_t blocks = (nwin + tpb - 1) / tpb;
  // a dispatch holds at most 2^32 - 1 work-items per dimension
  const uint64_t gx = std::min<uint64_t>(blocks, 0xFFFFFFFFull / tpb);
  const uint64_t gy = (blocks + gx - 1) / gx;
  if (gy > 65535) return set_err(ctx, RK_EUNSUPPORTED, "text too long for one paper-mode launch");
  *grid = dim3((uint32_t)gx, (uint32_t)gy, 1);
  return RK_OK;
}

}  // namespace rk

using namespace rk;

extern "C" rk_status rk_paper_search(rk_ctx *ctx, const uint8_t *text_dev, uint64_t n, const uint8_t *pattern_dev,
                                     const uint8_t *pattern_host, uint32_t m, uint32_t threads_per_block,
                                     uint8_t *result_dev, uint32_t *hash_dev, rk_stream s) {
  if (!ctx) return RK_EINVAL;
  if (m == 0) return set_err(ctx, RK_EINVAL, "m = 0");
  if (threads_per_block == 0 || threads_per_block > 1024)
    return set_err(ctx, RK_EINVAL, "threads per block must be 1..1024");
  if (n < m) return RK_OK;  // no window
  if (!text_dev || !pattern_dev || !pattern_host || !result_dev) return set_err(ctx, RK_EINVAL, "null pointer");
  const uint64_t nwin = n - m + 1;
  // the pattern's hash, once on the host (Sec. 3.1)
  uint32_t hx = 0;
  for (uint32_t i = 0; i < m; ++i) hx = (hx << 1) + pattern_host[i];
  dim3 grid;
  rk_status st = paper_grid(ctx, nwin, threads_per_block, &grid);
  if (st != RK_OK) return st;
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RK_EDEVICE, "hipSetDevice failed");
  hipStream_t hs = (hipStream_t)s;
  int slot = -1;
  hipError_t e = prof_begin(ctx, hs, 5, &slot);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(paper_kernel, grid, dim3(threads_per_block), 0, hs, text_dev, nwin, pattern_dev, m, hx,
                       result_dev, hash_dev);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = prof_end(ctx, hs, slot);
  return e == hipSuccess ? RK_OK : hip_err(ctx, e, "paper-mode launch");
}

extern "C" rk_status rk_paper_scratch_size(uint64_t nflags, uint64_t *bytes) {
  if (!bytes) return RK_EINVAL;
  const uint64_t nb = (nflags + kFlagBlock - 1) / kFlagBlock;
  *bytes = (nb * 4 + 255) / 256 * 256 + (nb * 8 + 255) / 256 * 256 + scan_tmp_words(nb) * 8 + 256;
  return RK_OK;
}

extern "C" rk_status rk_paper_positions(rk_ctx *ctx, const uint8_t *flags_dev, uint64_t nflags, void *scratch_dev,
                                        uint64_t scratch_bytes, uint64_t *positions_dev, uint64_t capacity,
                                        uint64_t *total_host, rk_stream s) {
  if (!ctx || !total_host) return RK_EINVAL;
  *total_host = 0;
  if (nflags == 0) return RK_OK;
  if (!flags_dev || !scratch_dev) return set_err(ctx, RK_EINVAL, "null pointer");
  uint64_t need = 0;
  rk_paper_scratch_size(nflags, &need);
  if (scratch_bytes < need) return set_err(ctx, RK_ENOSPACE, "scratch needs %llu bytes", (unsigned long long)need);
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RK_EDEVICE, "hipSetDevice failed");
  hipStream_t hs = (hipStream_t)s;
  const uint64_t nb = (nflags + kFlagBlock - 1) / kFlagBlock;
  uint8_t *sc = (uint8_t *)scratch_dev;
  uint32_t *counts = (uint32_t *)sc;
  uint64_t *offs = (uint64_t *)(sc + (nb * 4 + 255) / 256 * 256);
  uint64_t *tmp = (uint64_t *)((uint8_t *)offs + (nb * 8 + 255) / 256 * 256);
  uint64_t *total_dev = (uint64_t *)((uint8_t *)tmp + scan_tmp_words(nb) * 8);
  hipLaunchKernelGGL(flag_counts, dim3((uint32_t)nb), dim3(kFlagWG), 0, hs, flags_dev, nflags, counts);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_exclusive_scan(counts, nb, offs, tmp, total_dev, hs);
  if (e == hipSuccess) e = hipMemcpyAsync(ctx->pinned, total_dev, 8, hipMemcpyDeviceToHost, hs);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  if (e != hipSuccess) return hip_err(ctx, e, "paper positions count");
  const uint64_t total = ctx->pinned[0];
  *total_host = total;
  if (total > capacity) return set_err(ctx, RK_ENOSPACE, "positions capacity %llu < %llu matches",
                                       (unsigned long long)capacity, (unsigned long long)total);
  if (total == 0) return RK_OK;
  if (!positions_dev) return set_err(ctx, RK_EINVAL, "null positions");
  hipLaunchKernelGGL(flag_positions, dim3((uint32_t)nb), dim3(kFlagWG), 0, hs, flags_dev, nflags, offs, positions_dev);
  e = hipGetLastError();
  return e == hipSuccess ? RK_OK : hip_err(ctx, e, "paper positions launch");
}
