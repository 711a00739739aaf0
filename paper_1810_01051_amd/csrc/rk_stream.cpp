// Searches of texts that live in host memory or in a file, of any length
// (larger than device memory): the text goes to the device in pieces through
// two device buffers, each piece a one-text search with the plan's kernels.
//
// Piece i owns the windows starting in [i L, (i + 1) L) and holds the text
// bytes [i L, (i + 1) L + m_max - 1) (cut at n), where L = piece bytes -
// (m_max - 1): the same front/back overlap rule as tiles inside a search, so
// every window lies wholly inside the piece that owns it.  A piece's per-
// pattern lists come back ascending; positions at or past L belong to the
// next piece and are dropped; the rest are shifted by i L and appended, so the
// concatenation per pattern stays ascending.
//
// Overlap: piece i + 1 is staged into pinned host memory (up to 16 threads
// copy, or read from the file) while piece i is copied to the device and
// searched; the host-to-device copy of piece i + 1 runs on a copy stream
// while the collect of piece i runs on the search stream.  The link
// (host-to-device bandwidth) bounds the whole search.
#include <hip/hip_runtime.h>

#include <fcntl.h>
#include <sched.h>
#include <unistd.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "../../include/rk.h"
#include "rk_internal.h"
#include "rk_runtime.h"

namespace rk {

namespace {

struct DevMem {
  void *p = nullptr;
  uint64_t bytes = 0;
  ~DevMem() {
    if (p) hipFree(p);
  }
  hipError_t ensure(uint64_t b) {
    if (b <= bytes && p) return hipSuccess;
    if (p) hipFree(p);
    p = nullptr;
    bytes = 0;
    const hipError_t e = hipMalloc(&p, std::max<uint64_t>(b, 256));
    if (e == hipSuccess) bytes = std::max<uint64_t>(b, 256);
    return e;
  }
};

struct Pinned {
  uint8_t *p = nullptr;
  ~Pinned() {
    if (p) hipHostFree(p);
  }
};

// The source of the text: host memory or a file descriptor.
struct Source {
  const uint8_t *mem = nullptr;
  int fd = -1;
  uint64_t n = 0;
};

// Copies text bytes [off, off + len) of src into dst with up to `threads`
// threads (memcpy from host memory, pread from the file).  Returns false on a
// read error or a short file.
static bool stage(const Source &src, uint64_t off, uint64_t len, uint8_t *dst, int threads) {
  const uint64_t per = std::max<uint64_t>(1 << 22, (len + threads - 1) / threads);
  std::vector<std::thread> th;
  std::vector<char> ok((len + per - 1) / per + 1, 1);
  uint64_t idx = 0;
  for (uint64_t a = 0; a < len; a += per, ++idx) {
    const uint64_t b = std::min(len, a + per);
    auto job = [&, a, b, idx]() {
      if (src.mem) {
        memcpy(dst + a, src.mem + off + a, b - a);
        return;
      }
      uint64_t done = a;
      while (done < b) {
        const ssize_t r = pread(src.fd, dst + done, b - done, (off_t)(off + done));
        if (r <= 0) {
          ok[idx] = 0;
          return;
        }
        done += (uint64_t)r;
      }
    };
    if (b == len && th.empty()) job();
    else th.emplace_back(job);
  }
  for (auto &t : th) t.join();
  for (char c : ok)
    if (!c) return false;
  return true;
}

// Threads that stage a piece: the CPUs this process may run on, at most 16.
// Staging from pageable memory is a host memcpy that one thread runs at a
// fraction of the host's memory bandwidth; with 8 threads it took longer than
// the host-to-device copy of the same piece.
static int staging_threads() {
  cpu_set_t set;
  int n = 0;
  if (sched_getaffinity(0, sizeof set, &set) == 0) n = CPU_COUNT(&set);
  if (n <= 0) n = (int)std::thread::hardware_concurrency();
  return std::max(1, std::min(16, n));
}

struct PieceOut {
  std::vector<uint64_t> off;  // k + 1, after dropping positions >= L
  std::vector<uint64_t> pos;  // shifted to text positions
};

static rk_status run_pieces(rk_ctx *ctx, const rk_plan *plan, const Source &src, uint64_t piece_bytes,
                            rk_host_result **out) {
  const uint64_t n = src.n;
  const uint32_t k = plan->k_total;
  const uint64_t ov = plan->max_m ? plan->max_m - 1 : 0;
  if (piece_bytes < (1u << 16) || piece_bytes <= 2 * ov)
    return set_err(ctx, RK_EINVAL, "piece bytes %llu too small (at least 64 KiB and 2 (m_max - 1))",
                   (unsigned long long)piece_bytes);
  piece_bytes = (piece_bytes + 15) & ~15ull;
  const uint64_t L = piece_bytes - ov;
  const uint64_t npieces = n == 0 ? 0 : (n + L - 1) / L;
  if (hipSetDevice(ctx->device) != hipSuccess) return set_err(ctx, RK_EDEVICE, "hipSetDevice failed");
  DevMem text[2], scratch, work, offs, pos;
  Pinned pin[2];
  hipStream_t cs = nullptr, ss = nullptr;
  hipEvent_t copied[2] = {nullptr, nullptr}, used[2] = {nullptr, nullptr};
  rk_status st = RK_OK;
  std::vector<PieceOut> pieces;
  const int threads = staging_threads();
  auto fail = [&](hipError_t e, const char *what) { return hip_err(ctx, e, what); };
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&ss, hipStreamNonBlocking);
  for (int b = 0; b < 2 && e == hipSuccess; ++b) {
    e = hipEventCreateWithFlags(&copied[b], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&used[b], hipEventDisableTiming);
    if (e == hipSuccess) e = text[b].ensure(piece_bytes);
    if (e == hipSuccess) e = hipHostMalloc((void **)&pin[b].p, piece_bytes, hipHostMallocDefault);
  }
  uint64_t sb = 0;
  if (e == hipSuccess) {
    st = rk_scratch_size(ctx, plan, piece_bytes, &sb);
    if (st == RK_OK) e = scratch.ensure(sb);
  }
  if (e == hipSuccess) e = offs.ensure((uint64_t)(k + 1) * 8);
  if (e != hipSuccess) st = fail(e, "streamed search setup");
  std::vector<uint64_t> hoff(k + 1);
  auto piece_len = [&](uint64_t i) { return std::min(n, i * L + piece_bytes) - i * L; };
  // uploads staged piece i from pin[i & 1] into text[i & 1] on the copy stream
  auto upload = [&](uint64_t i) -> hipError_t {
    const int b = (int)(i & 1);
    hipError_t e2 = hipStreamWaitEvent(cs, used[b], 0);  // the search of piece i - 2 is done with text[b]
    if (e2 == hipSuccess) e2 = hipMemcpyAsync(text[b].p, pin[b].p, piece_len(i), hipMemcpyHostToDevice, cs);
    if (e2 == hipSuccess) e2 = hipEventRecord(copied[b], cs);
    return e2;
  };
  if (st == RK_OK && npieces) {
    if (!stage(src, 0, piece_len(0), pin[0].p, threads)) st = set_err(ctx, RK_EINVAL, "reading the text failed");
    else if ((e = upload(0)) != hipSuccess) st = fail(e, "piece upload");
  }
  for (uint64_t i = 0; i < npieces && st == RK_OK; ++i) {
    const int b = (int)(i & 1);
    const uint64_t a = i * L, len = piece_len(i);
    // piece i + 1 is staged on the host while piece i is searched: its pinned
    // buffer was last read by the upload of piece i - 1, which piece i - 1's
    // search waited for
    bool staged = true;
    std::thread stager;
    if (i + 1 < npieces)
      stager = std::thread([&, i]() { staged = stage(src, (i + 1) * L, piece_len(i + 1), pin[(i + 1) & 1].p, threads); });
    auto join = [&]() {
      if (stager.joinable()) stager.join();
    };
    e = hipStreamWaitEvent(ss, copied[b], 0);
    if (e != hipSuccess) {
      join();
      st = fail(e, "piece upload");
      break;
    }
    uint64_t total = 0;
    st = rk_count(ctx, plan, (const uint8_t *)text[b].p, len, scratch.p, sb, nullptr, &total, ss);
    uint64_t wb = 0;
    if (st == RK_OK) {
      rk_work_size(ctx, plan, total, &wb);
      e = work.ensure(wb);
      if (e == hipSuccess) e = pos.ensure(std::max<uint64_t>(total, 1) * 8);
      if (e != hipSuccess) st = set_err(ctx, RK_ENOMEM, "device memory for %llu hits of a piece", (unsigned long long)total);
    }
    if (st == RK_OK)
      st = rk_collect(ctx, plan, (const uint8_t *)text[b].p, len, scratch.p, sb, work.p, wb, (uint64_t *)offs.p,
                      (uint64_t *)pos.p, total, ss);
    std::vector<uint64_t> raw(total);
    if (st == RK_OK) {
      e = hipEventRecord(used[b], ss);
      if (e == hipSuccess) e = hipMemcpyAsync(hoff.data(), offs.p, (k + 1) * 8, hipMemcpyDeviceToHost, ss);
      if (e == hipSuccess && total) e = hipMemcpyAsync(raw.data(), pos.p, total * 8, hipMemcpyDeviceToHost, ss);
      if (e == hipSuccess) e = hipStreamSynchronize(ss);
      if (e != hipSuccess) st = fail(e, "piece results");
    }
    join();
    if (st != RK_OK) break;
    if (!staged) {
      st = set_err(ctx, RK_EINVAL, "reading text bytes from %llu failed", (unsigned long long)((i + 1) * L));
      break;
    }
    if (i + 1 < npieces && (e = upload(i + 1)) != hipSuccess) {
      st = fail(e, "piece upload");
      break;
    }
    // keep the windows this piece owns (start < L unless it is the last piece)
    const bool last = i + 1 == npieces;
    PieceOut po;
    po.off.assign(k + 1, 0);
    po.pos.reserve(total);
    for (uint32_t j = 0; j < k; ++j) {
      const uint64_t *s0 = raw.data() + hoff[j], *s1 = raw.data() + hoff[j + 1];
      const uint64_t *cut = last ? s1 : std::lower_bound(s0, s1, L);
      for (const uint64_t *q = s0; q < cut; ++q) po.pos.push_back(*q + a);
      po.off[j + 1] = po.pos.size();
    }
    pieces.push_back(std::move(po));
  }
  if (ss) hipStreamSynchronize(ss);
  if (cs) hipStreamSynchronize(cs);
  for (int b = 0; b < 2; ++b) {
    if (copied[b]) hipEventDestroy(copied[b]);
    if (used[b]) hipEventDestroy(used[b]);
  }
  if (cs) hipStreamDestroy(cs);
  if (ss) hipStreamDestroy(ss);
  if (st != RK_OK) return st;
  // per pattern: the pieces' lists in piece order
  uint64_t total = 0;
  for (const PieceOut &po : pieces) total += po.pos.size();
  rk_host_result *r = new (std::nothrow) rk_host_result();
  if (!r) return set_err(ctx, RK_ENOMEM, "result");
  r->k = k;
  r->total = total;
  r->offsets = new (std::nothrow) uint64_t[k + 1];
  r->positions = new (std::nothrow) uint64_t[std::max<uint64_t>(total, 1)];
  if (!r->offsets || !r->positions) {
    rk_host_result_free(r);
    return set_err(ctx, RK_ENOMEM, "result of %llu positions", (unsigned long long)total);
  }
  uint64_t o = 0;
  for (uint32_t j = 0; j < k; ++j) {
    r->offsets[j] = o;
    for (const PieceOut &po : pieces) {
      const uint64_t c = po.off[j + 1] - po.off[j];
      if (c) memcpy(r->positions + o, po.pos.data() + po.off[j], c * 8);
      o += c;
    }
  }
  r->offsets[k] = o;
  *out = r;
  return RK_OK;
}

}  // namespace

}  // namespace rk

using namespace rk;

extern "C" rk_status rk_search_host(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text_host, uint64_t n,
                                    uint64_t piece_bytes, rk_host_result **out) {
  if (!ctx || !plan || !out) return RK_EINVAL;
  *out = nullptr;
  if (plan->batch) return set_err(ctx, RK_EINVAL, "streamed searches take single-text plans");
  if (n && !text_host) return set_err(ctx, RK_EINVAL, "null text");
  Source src;
  src.mem = text_host;
  src.n = n;
  return run_pieces(ctx, plan, src, piece_bytes, out);
}

extern "C" rk_status rk_search_file(rk_ctx *ctx, const rk_plan *plan, const char *path, uint64_t piece_bytes,
                                    rk_host_result **out) {
  if (!ctx || !plan || !out || !path) return RK_EINVAL;
  *out = nullptr;
  if (plan->batch) return set_err(ctx, RK_EINVAL, "streamed searches take single-text plans");
  const int fd = open(path, O_RDONLY);
  if (fd < 0) return set_err(ctx, RK_EINVAL, "cannot open %s", path);
  const off_t end = lseek(fd, 0, SEEK_END);
  if (end < 0) {
    close(fd);
    return set_err(ctx, RK_EINVAL, "cannot size %s", path);
  }
  Source src;
  src.fd = fd;
  src.n = (uint64_t)end;
  const rk_status st = run_pieces(ctx, plan, src, piece_bytes, out);
  close(fd);
  return st;
}

extern "C" void rk_host_result_free(rk_host_result *r) {
  if (!r) return;
  delete[] r->offsets;
  delete[] r->positions;
  delete r;
}
