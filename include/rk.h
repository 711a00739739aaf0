/*
 * rk.h -- C ABI of librk, an MI355X (gfx950) multi-pattern Rabin-Karp search.
 *
 * Problem (Shah & Oza, "Improved Parallel Rabin-Karp Algorithm Using CUDA",
 * Sec. 1 and Sec. 3.1): find every occurrence of every pattern P_j in a text T.
 * For each text window the library forms a polynomial hash, tests it against the
 * set of pattern hashes and confirms a hit by comparing bytes, as the paper's
 * sequential and GPU procedures do for one pattern.
 *
 *   hash(s[0..m)) = sum_{i<m} s[i] * d^(m-1-i)  (mod q),   bytes unsigned,
 *
 * with d = 256 and q = 2^61 - 1 fixed by this library (the paper's own hash is
 * the shift-and-add case d = 2 with no modulus).  Results are exact: pattern j's
 * result is the ascending list of every x in [0, n - m_j] with
 * T[x .. x+m_j) == P_j, overlapping occurrences included, whatever hash
 * collisions happen.
 *
 * Conventions for every call:
 *   - No call throws or aborts; each returns an rk_status.  After a non-OK
 *     status rk_ctx_last_error() describes it and outputs are undefined.
 *   - "_dev" pointers are device memory of the context's GPU; "_host" pointers
 *     are host memory.  The caller owns every buffer it passes; the library
 *     never frees or modifies inputs and keeps no pointer to them after the call
 *     returns, except where a call says otherwise (plans and servers keep the
 *     device text pointers they are given until destroyed).
 *   - Text device pointers must be 16-byte aligned (RK_EINVAL otherwise): the
 *     scan reads whole aligned 16-byte blocks, so it never touches a block that
 *     holds no text byte.
 *   - rk_stream is a hipStream_t (NULL: the legacy default stream).  Work is
 *     enqueued on it; calls that return a host-visible value synchronise it.
 *   - A context is bound to one device and is not thread-safe; use one per
 *     host thread.  The server object is the exception (see below).
 *   - Pattern lengths: 1 <= m <= RK_MAX_M.  m = 0 is RK_EINVAL, m > RK_MAX_M is
 *     RK_EUNSUPPORTED, m > n yields an empty list.  k = 0 is valid (no hits).
 *   - Device faults and launch failures surface as RK_EDEVICE.
 */
#ifndef RK_H
#define RK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RK_MAX_M 1024u               /* longest pattern (windows longer than RK_STREAM_M are tested by
                                        their last RK_STREAM_M bytes, then byte-checked whole) */
#define RK_STREAM_M 64u              /* longest window a scan hashes by rolling */
#define RK_MAX_PID ((1u << 24) - 1)  /* largest pattern id in one plan (k <= 2^24) */
#define RK_MAX_N ((1ull << 40) - 1)  /* largest text length (positions are 40-bit) */

typedef enum {
  RK_OK = 0,
  RK_EINVAL = -1,       /* bad argument: null pointer, m = 0, misaligned text, ... */
  RK_ENOMEM = -2,       /* host or device allocation failed */
  RK_EUNSUPPORTED = -3, /* valid but not supported: d or q other than 256 / 2^61-1, m > RK_MAX_M */
  RK_EDEVICE = -4,      /* HIP runtime error or device fault */
  RK_ENOSPACE = -5,     /* a caller buffer (scratch, work, output capacity) is too small */
  RK_EBUSY = -6,        /* request not finished yet (server poll) */
  RK_ECANCELED = -7,    /* request canceled or its server shut down */
  RK_ETIMEDOUT = -8     /* request waited longer than the server's request timeout */
} rk_status;

/* Scan modes.  Both give identical results.
 *   RK_MODE_EXACT : every window's d=256 / q=2^61-1 hash is rolled and tested
 *                   against the pattern-hash set; equal hashes are byte-checked.
 *                   A set whose lengths all agree (one pattern, say) hashes
 *                   whole windows.  Several lengths share one stream per
 *                   length class (1, 2, 3, 4..7, 8..15, 16..31, 32 and more):
 *                   it hashes the last l bytes of every window, l the shortest
 *                   length of the class (at most RK_STREAM_M), and each
 *                   pattern is keyed by the hash of its last l bytes.
 *   RK_MODE_SCREEN: every window gets a shift-and-add hash in the paper's form
 *                   h <- (h << s) + c taken mod 2^32 (the polynomial hash
 *                   with d = 2^s, q = 2^32) with s = 8 for patterns shorter
 *                   than 8 bytes (masked to the window below 4), 4 for 8..15
 *                   and 2 from 16 (so the hash covers the last 32/s bytes of
 *                   a window: every pattern of 16 bytes or more shares one
 *                   stream), tested against the set of the patterns' shift-add
 *                   hashes; windows in the set are byte-checked against the
 *                   patterns with that hash (the byte check stands in for the
 *                   exact hash, which can only pass what the bytes pass).  A
 *                   true occurrence always passes the test, so no occurrence
 *                   is lost.  The paper's own s = 1 over whole windows is
 *                   rk_paper_search.
 *   RK_MODE_AUTO  : RK_MODE_SCREEN. */
typedef enum { RK_MODE_AUTO = 0, RK_MODE_EXACT = 1, RK_MODE_SCREEN = 2 } rk_mode;

typedef void *rk_stream; /* hipStream_t */

typedef struct rk_ctx rk_ctx;
typedef struct rk_plan rk_plan;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device` for base d and modulus q (the
 * parameters of the polynomial hash of Sec. 3.1; the paper's own are d = 2
 * with no modulus, see rk_paper_search).  Only
 * d = 256 and q = 2^61 - 1 are supported (RK_EUNSUPPORTED otherwise); the
 * arguments exist so that the hash parameters are explicit at the boundary.
 * *out receives the context.  Makes `device` current on the calling thread. */
rk_status rk_ctx_create(int device, uint64_t d, uint64_t q, rk_ctx **out);
void rk_ctx_destroy(rk_ctx *ctx);
/* Text of the last failure on this context ("" if none).  Owned by the context. */
const char *rk_ctx_last_error(const rk_ctx *ctx);
/* Static name of a status code. */
const char *rk_status_string(rk_status s);

/* Options (rk_ctx_set_option).  Values are read when a plan is created or a
 * scan is launched. */
typedef enum {
  RK_OPT_SLAB_CAP = 1,  /* per-tile staging slots for hits (0 = default: tile bytes / 64 for
                           one pattern, / 16 for pattern sets).  Tiles with more hits are
                           rescanned by rk_collect. */
  RK_OPT_TILE_CFG = 2,  /* scan geometry index into the built-in table (see rk_tile_cfg);
                           -1 = autotuned / default */
  RK_OPT_GRID = 3,      /* workgroups of the scan, which strides over the tiles (0 = default:
                           32 times as many as are resident on every CU at once for the
                           single-pattern scan, as many as are resident for the others) */
  RK_OPT_PROFILE = 4,   /* 1: time every scan launch with HIP events (rk_ctx_profile) */
  RK_OPT_QUEUE = 5      /* 1: scan pulls tiles from an atomic work queue; 0: static striding;
                           -1 (default): queue for multi-instance plans only */
} rk_option;
rk_status rk_ctx_set_option(rk_ctx *ctx, int option, int64_t value);

/* Scan geometry table entry i (0 <= i < rk_tile_cfg_count()): workgroup size,
 * windows per thread, and tile bytes = wg * windows. */
int rk_tile_cfg_count(void);
rk_status rk_tile_cfg(int i, uint32_t *wg, uint32_t *windows_per_thread, uint32_t *tile_bytes);

/* Accumulated device time of scan launches since profiling was switched on.
 * kernel: 0 = scan (count pass), 1 = rescan of overflowed tiles, 2 = collect
 * (compaction + sort), 3 = all of 0..2, 4 = rk_stream_read, 5 = rk_paper_search.
 * Synchronises the context's device. */
rk_status rk_ctx_profile(rk_ctx *ctx, int kernel, uint64_t *launches, double *total_ms);
rk_status rk_ctx_profile_reset(rk_ctx *ctx);

/* hash(s[0..m)) in [0, q), computed on the host with the library's own
 * arithmetic (Sec. 3.1: the pattern hash hx is computed once on the host). */
rk_status rk_hash(const rk_ctx *ctx, const uint8_t *s_host, uint64_t m, uint64_t *out);

/* -------------------------------------------------------------------- plans */

/* A plan holds preprocessed patterns (the paper computes hx once on the host and
 * passes it to the kernel, Sec. 3.1): lengths bucketed, pattern hashes and
 * screen hashes computed, per-bucket hash tables built and uploaded.
 * Pattern j = bytes_host[offsets_host[j] .. offsets_host[j+1]), j < k; the
 * host arrays are copied and may be freed after the call.  mode: rk_mode. */
rk_status rk_plan_create(rk_ctx *ctx, const uint8_t *bytes_host, const uint64_t *offsets_host,
                         uint32_t k, int mode, rk_plan **out);
void rk_plan_destroy(rk_plan *plan);
/* Number of patterns (for a batch plan: the sum over instances). */
uint32_t rk_plan_patterns(const rk_plan *plan);

/* Bytes of device scratch that rk_count / rk_collect need for a text of n
 * (per-tile staging of hits, which replaces the dense result array of
 * Sec. 3.1)
 * bytes (a function of n, the plan and RK_OPT_SLAB_CAP). */
rk_status rk_scratch_size(rk_ctx *ctx, const rk_plan *plan, uint64_t n, uint64_t *bytes);

/* Count pass (the first half of Sec. 1's problem, "find all occurrences":
 * every window of Sec. 3.1's GPU procedure hashed, tested against the set and
 * byte-checked): scans text_dev[0..n) once, stages hits in scratch_dev and
 * writes the number of hits over all patterns to *total_host.  counts_dev
 * (optional, NULL to skip): k entries (u64, device), pattern j's number of
 * occurrences.  Synchronises s.  scratch must hold rk_scratch_size bytes
 * (RK_ENOSPACE otherwise) and must be passed unchanged to the rk_collect that
 * follows. */
rk_status rk_count(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text_dev, uint64_t n,
                   void *scratch_dev, uint64_t scratch_bytes, uint64_t *counts_dev, uint64_t *total_host,
                   rk_stream s);

/* Bytes of device work memory rk_collect needs when the count was `total`
 * (0 for single-pattern plans). */
rk_status rk_work_size(rk_ctx *ctx, const rk_plan *plan, uint64_t total, uint64_t *bytes);

/* Collect pass (the second half of Sec. 1's problem: the occurrences
 * themselves, in place of the GPU procedure's dense result array of Sec. 3.1),
 * after rk_count with the same plan, text and scratch: writes
 * offsets_dev[0..k] (offsets_dev[j+1] - offsets_dev[j] = hits of pattern j,
 * offsets_dev[0] = 0) and positions_dev[offsets[j] .. offsets[j+1]) = pattern
 * j's positions, strictly ascending.  capacity = entries of positions_dev
 * (RK_ENOSPACE if below the total).  Does not synchronise s. */
rk_status rk_collect(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text_dev, uint64_t n,
                     void *scratch_dev, uint64_t scratch_bytes, void *work_dev, uint64_t work_bytes,
                     uint64_t *offsets_dev, uint64_t *positions_dev, uint64_t capacity, rk_stream s);

/* Window hashes (Sec. 3.1: the hash hy of the substring at offset x, here
 * with d = 256, q = 2^61 - 1):
 * out_dev[i] = hash(text_dev[xs_dev[i] .. xs_dev[i]+m)) in [0, q),
 * each evaluated directly (Horner) on the device.  Every xs_dev[i] must satisfy
 * xs + m <= n; out-of-range entries get the value UINT64_MAX. */
rk_status rk_window_hashes(rk_ctx *ctx, const uint8_t *text_dev, uint64_t n, uint32_t m,
                           const uint64_t *xs_dev, uint64_t cnt, uint64_t *out_dev, rk_stream s);

/* Hash dump of the scan itself (the "identical window hashes on sampled
 * dumps" check of the exact path): runs an exact-mode scan kernel for length m
 * over text_dev[0..n) and writes, from the rolling state of its own hash loop
 * (the same initial state, rolling step and out-stream as its pattern test),
 * the canonical hash of window x = i * stride to out_dev[i] for
 * i < cnt = floor((n - m) / stride) + 1, for 1 <= m <= RK_STREAM_M
 * (RK_EUNSUPPORTED above: longer patterns are tested by the hash of their
 * last RK_STREAM_M bytes).  kernel 0: the general scan kernel
 * (pattern sets, batches); 1: the single-bucket kernel that one-pattern
 * searches run.  The geometry is RK_OPT_TILE_CFG's, else the autotuned one
 * for (exact, m).  cap = entries of out_dev (RK_ENOSPACE if below cnt).
 * Synchronises s.  (Sec. 3.1: the window hash of every offset.) */
rk_status rk_scan_dump(rk_ctx *ctx, const uint8_t *text_dev, uint64_t n, uint32_t m,
                       uint64_t stride, uint64_t *out_dev, uint64_t cap, int kernel, rk_stream s);

/* Read-bandwidth ceiling for the scan's roofline: reads data_dev[0..n) once
 * the way the scans load their tiles (non-temporal 16-byte loads straight into
 * LDS, 1 KiB per wave load, grid workgroups of 256 threads, grid-stride) and
 * writes the XOR fold of each workgroup's words to out_dev[0..grid).
 * data_dev 16-byte aligned, n a multiple of 16.  Timed by RK_OPT_PROFILE as
 * kernel 4. */
rk_status rk_stream_read(rk_ctx *ctx, const void *data_dev, uint64_t n, uint32_t *out_dev, uint32_t grid,
                         rk_stream s);

/* ------------------------------------------------ search without allocation */

/* Largest scratch + work memory rk_search_static can use (bytes): the size of
 * the library's static device array, of which each GPU holds one copy from
 * load until the process ends. */
#define RK_STATIC_SCRATCH_BYTES (64ull << 20)

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): rk_count followed by
 * rk_collect with their scratch and work memory taken from the library's
 * static device array instead of caller buffers.  No hipMalloc, hipFree or
 * other allocation happens in the call.  The caller passes the text and the
 * outputs (offsets_dev: k + 1 entries, positions_dev: capacity entries, as for
 * rk_collect); *total_host receives the number of hits.  Returns RK_ENOSPACE
 * (with the reason in rk_ctx_last_error) when the count's scratch or the
 * collect's work memory would exceed RK_STATIC_SCRATCH_BYTES, or when
 * capacity is below the total (then *total_host is set and nothing is
 * written).  Synchronises s once (after the count).  Every call on one GPU
 * shares that GPU's array and leaves its contents behind: calls that overlap
 * on one GPU (other streams or host threads) race and must be serialised by
 * the caller. */
rk_status rk_search_static(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text_dev, uint64_t n,
                           uint64_t *offsets_dev, uint64_t *positions_dev, uint64_t capacity,
                           uint64_t *total_host, rk_stream s);
/* RK_STATIC_SCRATCH_BYTES as built into the library. */
uint64_t rk_static_scratch_bytes(void);

/* ------------------------------------------- texts in host memory or a file */

/* Result of a streamed search, in host memory owned by the library: pattern
 * j's ascending positions are positions[offsets[j] .. offsets[j+1]). */
typedef struct {
  uint32_t k;
  uint64_t total;
  uint64_t *offsets;    /* k + 1 entries */
  uint64_t *positions;  /* total entries */
} rk_host_result;

/* Search of a text that lives in host memory (text_host, n bytes, any
 * alignment, pageable) -- of any length, device memory holding only two
 * pieces of piece_bytes (rounded up to 16; at least 64 KiB and twice the
 * longest pattern).  The paper reads T and P from files and moves them to the
 * device (Sec. 3.1); here the text moves piece by piece: piece i owns the
 * windows starting in [i L, (i+1) L), L = piece_bytes - (m_max - 1), and holds
 * the m_max - 1 bytes after them, so each window is searched in exactly one
 * piece.  Staging of the next piece (host threads), its host-to-device copy
 * and the search of the current one overlap.  plan: a single-text plan (not a
 * batch).  *out receives the result (free with rk_host_result_free).
 * Allocates device memory for the pieces, scratch and each piece's hits. */
rk_status rk_search_host(rk_ctx *ctx, const rk_plan *plan, const uint8_t *text_host, uint64_t n,
                         uint64_t piece_bytes, rk_host_result **out);
/* The same for the bytes of the file at path (read with pread, piece by piece). */
rk_status rk_search_file(rk_ctx *ctx, const rk_plan *plan, const char *path, uint64_t piece_bytes,
                         rk_host_result **out);
void rk_host_result_free(rk_host_result *r);

/* ------------------------------------------------------- paper-faithful mode */

/* The paper's GPU procedure as printed (Sec. 3.1), for rerunning its
 * experiments (Tables 1-3: threads per block, pattern length) next to the
 * tiled scans: one thread per offset x in [0, n - m] (grid of
 * ceil((n - m + 1) / threads_per_block) blocks of threads_per_block threads,
 * 1..1024), each hashing the m bytes at text_dev + x with h <- (h << 1) + c in
 * a 32-bit word (d = 2, q = 2^32) read straight from device memory, comparing
 * with the pattern's hash (computed here on the host from pattern_host) and,
 * on equality, comparing the m bytes with pattern_dev.  result_dev[x] = 1 for
 * a match, 0 otherwise (n - m + 1 bytes, the paper's result array).  hash_dev
 * (optional, NULL to skip): n - m + 1 u32, every window's hash.  Any m >= 1;
 * m > n launches nothing.  text_dev needs no alignment.  Asynchronous on s;
 * timed by RK_OPT_PROFILE as kernel 5. */
rk_status rk_paper_search(rk_ctx *ctx, const uint8_t *text_dev, uint64_t n, const uint8_t *pattern_dev,
                          const uint8_t *pattern_host, uint32_t m, uint32_t threads_per_block,
                          uint8_t *result_dev, uint32_t *hash_dev, rk_stream s);
/* Device scratch bytes rk_paper_positions needs for nflags result bytes. */
rk_status rk_paper_scratch_size(uint64_t nflags, uint64_t *bytes);
/* Ascending positions of the nonzero bytes of flags_dev[0..nflags) (a result
 * array of rk_paper_search) into positions_dev (capacity entries; RK_ENOSPACE
 * if fewer than the count, which *total_host still receives).  Synchronises s
 * once (for the count). */
rk_status rk_paper_positions(rk_ctx *ctx, const uint8_t *flags_dev, uint64_t nflags, void *scratch_dev,
                             uint64_t scratch_bytes, uint64_t *positions_dev, uint64_t capacity,
                             uint64_t *total_host, rk_stream s);

/* ----------------------------------------------------------------- batching */

/* One search instance of a batch: text on the device (16-byte aligned), its
 * patterns on the host (same layout as rk_plan_create). */
typedef struct {
  const uint8_t *text_dev;
  uint64_t n;
  const uint8_t *bytes_host;
  const uint64_t *offsets_host;
  uint32_t k;
} rk_instance;

/* Plan for `count` independent searches (each the problem of Sec. 1 on its
 * own text; the paper runs one search per launch, Sec. 3.1) scanned by
 * persistent launches (one per scan geometry in use), each over an atomic
 * work queue of (instance, tile) items.  Each instance's text is scanned once
 * for all its pattern-length buckets, with the geometry whose tuned bucket
 * timings (rk_autotune / rk_autotune_load) sum to the least over the
 * instance's buckets.  Instance i's
 * patterns get global ids base_i + j with base_i = sum of k over instances
 * before i.  The plan keeps the text pointers; the texts must stay alive and
 * unchanged while the plan is used. */
rk_status rk_batch_plan_create(rk_ctx *ctx, const rk_instance *inst, uint32_t count, int mode,
                               rk_plan **out);
/* rk_count / rk_collect on a batch plan: text_dev must be NULL and n is the
 * total text bytes over instances (as passed to rk_scratch_size); offsets_dev
 * has (sum k) + 1 entries; positions are relative to each instance's text. */
uint64_t rk_plan_text_bytes(const rk_plan *plan);

/* ---------------------------------------------------------------- autotuner */

/* Times every scan geometry of the built-in table on a synthetic DNA text of
 * n bytes (n >= 64 KiB; byte i = "ACGT"[x_i >> 62] for Knuth's MMIX linear
 * congruential sequence x_{i+1} = 6364136223846793005 x_i + 1442695040888963407,
 * x_0 = 0x181001051):
 *   - for one pattern of each length in lengths (the text's bytes at n/3),
 *     both modes, the single-bucket kernel of one-pattern searches;
 *   - for each batch bucket (m-class 0..4: lengths 1-3, 4-7, 8-15, 16-31,
 *     32-64; k-class 0..3: 1, 4, 32, 256 patterns), both modes, the general
 *     kernel over a one-instance batch plan of the text's first n_b bytes
 *     (n_b = min(n, 1 MiB) for m-class 0, min(n, 32 MiB) otherwise), pattern j
 *     of length lo + j mod (hi - lo + 1) copied from the text at
 *     (n_b/3 + 7919 j) mod (n_b - m + 1), reversed when j is odd,
 * stores the fastest geometry of each and every bucket timing in the context
 * (a batch instance is scanned once, all its m-buckets together, with the
 * geometry of least tuned time summed over its buckets) and, if path is non-NULL,
 * writes the table as JSON with every candidate's time, hit count and digest
 * of its result (sum of v[i] * (2i + 1) mod 2^64 over the offsets followed by
 * the positions).  Every candidate must return the same hits (RK_EDEVICE otherwise).
 * Synchronises the device.  (The paper's Tables 1-2 vary threads per block
 * for the same reason: the launch shape decides the speed.) */
rk_status rk_autotune(rk_ctx *ctx, uint64_t n, const uint32_t *lengths, uint32_t nlengths,
                      const char *path);
/* Load a table written by rk_autotune (entries for another gfx arch are ignored). */
rk_status rk_autotune_load(rk_ctx *ctx, const char *path);
/* Geometry index the scan uses for (mode, pattern length m) of one-pattern searches. */
int rk_autotune_choice(const rk_ctx *ctx, int mode, uint32_t m);
/* Geometry index of a batch bucket (mode, m-class, k-class); -1 if not tuned. */
int rk_autotune_bucket_choice(const rk_ctx *ctx, int mode, int mclass, int kclass);

#ifdef __cplusplus
}
#endif
#endif /* RK_H */
