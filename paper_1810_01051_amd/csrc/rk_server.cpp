// Continuous-batching search server (include/rk_server.h).
//
// Client threads append requests to a queue.  One scheduler thread owns a
// private librk context and up to max_inflight stream slots.  For an idle
// slot it takes the oldest waiting request and the other waiting requests for
// the same corpus, in arrival order, and concatenates their patterns, each
// request's patterns getting consecutive ids of the merged set, so that its
// result is a contiguous slice of the merged output (no copy per request;
// identical patterns of one step share their bytes in the table image).  It
// builds a batch plan for the corpus and enqueues the count pass.  When a slot's count is done the step is admitted
// once the output arena can hold its hits; a step that could never fit is
// split and counted again, and a step that finds the arena held by unreleased
// results with nothing else in flight waits a bounded time, then fails.  Then the collect pass writes the sorted hits and
// the per-pattern offsets come back to pinned host memory.  Count and collect
// launches of each step are captured into a graph that updates the slot's
// executable graph in place (hipGraphExecUpdate; re-instantiated when the
// launch sequence changes) and launched as one unit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/rk.h"
#include "../../include/rk_server.h"
#include "rk_internal.h"
#include "rk_runtime.h"

namespace rk {

static inline uint64_t aup(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// Device block holding the merged positions of one step; the requests of the
// step own slices of it and the block goes back to the arena when the last of
// them is released.
struct StepBuf {
  uint64_t off = 0, size = 0;
  uint32_t refs = 0;
};

struct Request {
  uint64_t id = 0;
  uint32_t corpus = 0;
  uint32_t k = 0;
  std::vector<uint8_t> bytes;
  std::vector<uint64_t> offs;
  rk_status status = RK_EBUSY;
  std::vector<uint64_t> res_offsets;  // host, k+1
  uint64_t out_off = 0, out_size = 0; // the request's positions in the arena (bytes)
  StepBuf *buf = nullptr;             // block that holds them
  uint32_t gp0 = 0;                   // merged id of the request's first pattern in its step
  double t_submit = 0, t_start = 0, t_done = 0;
  uint64_t step = 0;
};

struct Corpus {
  const uint8_t *text;
  uint64_t n;
};

// First-fit allocator over [0, cap) in 256-byte units with coalescing.
struct Arena {
  uint64_t cap = 0, used = 0, high = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> size
  void init(uint64_t c) {
    cap = c;
    free_.clear();
    if (c) free_[0] = c;
    used = high = 0;
  }
  bool alloc(uint64_t size, uint64_t *off) {
    size = aup(std::max<uint64_t>(size, 256), 256);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= size) {
        *off = it->first;
        const uint64_t rest = it->second - size, at = it->first + size;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used += size;
        high = std::max(high, used);
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t size) {
    size = aup(std::max<uint64_t>(size, 256), 256);
    used -= size;
    auto it = free_.emplace(off, size).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

enum SlotState { kIdle, kCounting, kCounted, kCollecting };

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t ev_count = nullptr, ev_collect = nullptr;
  SlotState state = kIdle;
  rk_plan plan;
  void *dplan = nullptr;
  uint64_t dplan_cap = 0;
  void *scratch = nullptr;
  uint64_t scratch_cap = 0;
  uint8_t *hstage = nullptr;  // pinned: plan bytes for the upload
  uint64_t hstage_cap = 0;
  uint64_t *hres = nullptr;   // pinned: merged per-pattern offsets of the step
  uint64_t hres_cap = 0;      // bytes
  uint64_t *hctr = nullptr;   // pinned: total, overflow count
  hipGraphExec_t gcount = nullptr, gcollect = nullptr;
  std::vector<Request *> reqs;
  uint64_t step_id = 0, n_total = 0, total = 0, plan_bytes = 0;
  uint32_t ovf = 0;
  bool estimated = false;              // the step's hit rate entered the server's estimate
  uint32_t slab_cap = 0;               // staging records per tile of the step (0: the default)
  uint64_t pos_off = 0, pos_size = 0;  // merged positions of the step (arena)
  uint64_t aux_off = 0, aux_size = 0;  // per-pattern offsets and sort work (arena)
  double t_start = 0;
  double wait_since = 0;               // counted step waiting for arena space with nothing else in flight
};

static double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace rk

using namespace rk;

struct rk_server {
  rk_ctx *ctx = nullptr;  // private context, used by the scheduler thread only
  int device = 0;
  rk_server_cfg cfg;
  std::mutex mu;
  std::condition_variable cv_submit, cv_done;
  std::deque<Request *> pending;
  std::unordered_map<uint64_t, Request *> reqs;
  std::deque<uint64_t> done_q;  // finished requests in completion order, for rk_server_next_done
  std::vector<Corpus> corpora;
  uint64_t next_id = 1, next_step = 1;
  bool stop = false;
  std::thread th;
  void *arena_dev = nullptr;
  hipStream_t fetch_stream = nullptr;  // client copies of results (never the legacy stream)
  Arena arena;
  std::vector<Slot> slots;
  // statistics (under mu)
  std::vector<double> lat_ms;
  uint64_t submitted = 0, completed = 0, canceled = 0, failed = 0, steps = 0, bytes_scanned = 0;
  uint64_t merged_patterns = 0, request_patterns = 0, admission_waits = 0, step_splits = 0;
  uint32_t step_limit = 0;   // requests per step, lowered after a split and raised again
  double hits_per_pattern = -1;  // running estimate from counted steps (-1: none yet)
  double busy_s = 0, busy_since = 0;
  uint32_t inflight = 0;
  uint64_t outstanding = 0;  // submitted and not finished
};

namespace rk {

static void finish_request(rk_server *S, Request *r, rk_status st) {
  r->status = st;
  r->t_done = now_s();
  S->done_q.push_back(r->id);
  if (S->outstanding) --S->outstanding;
  if (st == RK_OK) {
    ++S->completed;
    S->lat_ms.push_back((r->t_done - r->t_submit) * 1e3);
    S->request_patterns += r->k;
  } else if (st == RK_ECANCELED) {
    ++S->canceled;
  } else {
    ++S->failed;
  }
}

// A failed allocation is RK_ENOMEM (the step can be retried smaller), any
// other HIP error RK_EDEVICE.
static rk_status alloc_err(rk_ctx *ctx, hipError_t e, const char *what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    return set_err(ctx, RK_ENOMEM, "%s: out of memory", what);
  }
  return hip_err(ctx, e, what);
}

static hipError_t ensure_dev(void **p, uint64_t *cap, uint64_t need) {
  if (need <= *cap && *p) return hipSuccess;
  if (*p) hipFree(*p);
  *p = nullptr;
  *cap = 0;
  const uint64_t c = aup(std::max<uint64_t>(need, 4096) * 5 / 4, 4096);
  hipError_t e = hipMalloc(p, c);
  if (e == hipSuccess) *cap = c;
  return e;
}

template <typename T>
static hipError_t ensure_pinned(T **p, uint64_t *cap, uint64_t need) {
  if (need <= *cap && *p) return hipSuccess;
  if (*p) hipHostFree(*p);
  *p = nullptr;
  *cap = 0;
  const uint64_t c = aup(std::max<uint64_t>(need, 4096) * 5 / 4, 4096);
  hipError_t e = hipHostMalloc((void **)p, c, hipHostMallocDefault);
  if (e == hipSuccess) *cap = c;
  return e;
}

static void drop_graphs(Slot &sl) {
  if (sl.gcount) hipGraphExecDestroy(sl.gcount);
  if (sl.gcollect) hipGraphExecDestroy(sl.gcollect);
  sl.gcount = sl.gcollect = nullptr;
}

// Runs enq() on the slot's stream, either directly or captured into a graph
// that replaces the slot's previous one (updated in place when it can be).
template <typename F>
static rk_status run_maybe_graph(rk_server *S, Slot &sl, hipGraphExec_t *exec, F &&enq) {
  if (!S->cfg.use_graphs) return enq();
  // relaxed: client threads keep making their own HIP calls while a step is
  // captured (the capturing thread makes no unsafe call inside enq)
  hipError_t e = hipStreamBeginCapture(sl.stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return hip_err(S->ctx, e, "begin capture");
  rk_status st = enq();
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(sl.stream, &g);
  if (st != RK_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return hip_err(S->ctx, e, "end capture");
  bool ok = false;
  if (*exec) {
    hipGraphNode_t err_node = nullptr;
    hipGraphExecUpdateResult res;
    ok = hipGraphExecUpdate(*exec, g, &err_node, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
    if (!ok) {
      (void)hipGetLastError();
      hipGraphExecDestroy(*exec);
      *exec = nullptr;
    }
  }
  if (!ok) {
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      hipGraphDestroy(g);
      return hip_err(S->ctx, e, "graph instantiate");
    }
  }
  hipGraphDestroy(g);
  e = hipGraphLaunch(*exec, sl.stream);
  if (e != hipSuccess) return hip_err(S->ctx, e, "graph launch");
  return RK_OK;
}

// Builds the step of an idle slot from the waiting requests (mu held on entry,
// released while the plan is built) and enqueues its count pass.
static rk_status start_step(rk_server *S, Slot &sl, std::unique_lock<std::mutex> &lk) {
  // take requests in arrival order
  std::vector<Request *> take;
  uint64_t pats = 0;
  // requests are also bounded by the output the step is expected to need:
  // about 20 bytes per hit (positions, sort buffer, histograms) at the hit
  // rate per pattern seen so far must fit the slot's share of the arena; the
  // first step, with no estimate yet, takes a few requests only
  uint32_t limit = std::min(S->cfg.max_step_requests, std::max<uint32_t>(S->step_limit, 1));
  if (S->hits_per_pattern < 0) limit = std::min<uint32_t>(limit, 8);
  const double share = (double)S->arena.cap / (double)S->slots.size();
  const double per_pat = S->hits_per_pattern < 0 ? 0.0 : 20.0 * S->hits_per_pattern;
  // A step serves one corpus: the oldest waiting request's, with the other
  // waiting requests for that corpus in arrival order (requests for other
  // corpora keep their places).  One corpus per step lets its requests share
  // the scan and keeps the merged pattern ids (and so the sort) small.
  const uint32_t corpus = S->pending.front()->corpus;
  std::deque<Request *> keep;
  while (!S->pending.empty() && take.size() < limit) {
    Request *r = S->pending.front();
    if (r->corpus == corpus) {
      if (!take.empty() && pats + r->k > S->cfg.max_step_patterns) break;
      if (!take.empty() && per_pat * (double)(pats + r->k) > share) break;
      take.push_back(r);
      pats += r->k;
    } else {
      keep.push_back(r);
    }
    S->pending.pop_front();
  }
  // the skipped requests go back in front, in their order
  for (auto it = keep.rbegin(); it != keep.rend(); ++it) S->pending.push_front(*it);
  const uint64_t step_id = S->next_step++;
  const double t0 = now_s();
  for (Request *r : take) {
    r->t_start = t0;
    r->step = step_id;
  }
  lk.unlock();
  // concatenate the requests' patterns per corpus: request i owns the merged
  // ids [gp0, gp0 + k) of its corpus instance
  struct CB {
    std::vector<uint8_t> bytes;
    std::vector<uint64_t> offs{0};
  };
  std::map<uint32_t, CB> by;
  std::vector<uint32_t> local(take.size());
  for (size_t i = 0; i < take.size(); ++i) {
    Request *r = take[i];
    CB &cb = by[r->corpus];
    local[i] = (uint32_t)(cb.offs.size() - 1);
    const uint64_t b0 = cb.bytes.size();
    cb.bytes.insert(cb.bytes.end(), r->bytes.begin(), r->bytes.end());
    for (uint32_t j = 0; j < r->k; ++j) cb.offs.push_back(b0 + r->offs[j + 1]);
  }
  std::vector<rk_instance> inst;
  std::map<uint32_t, uint32_t> base;
  uint32_t kt = 0;
  uint64_t nbytes = 0;
  for (auto &kv : by) {
    rk_instance I;
    I.text_dev = S->corpora[kv.first].text;
    I.n = S->corpora[kv.first].n;
    I.bytes_host = kv.second.bytes.data();
    I.offsets_host = kv.second.offs.data();
    I.k = (uint32_t)(kv.second.offs.size() - 1);
    base[kv.first] = kt;
    kt += I.k;
    nbytes += I.n;
    inst.push_back(I);
  }
  for (size_t i = 0; i < take.size(); ++i) take[i]->gp0 = base[take[i]->corpus] + local[i];
  // host plan
  sl.plan = rk_plan();
  std::vector<uint8_t> blob;
  std::vector<InstDesc> descs;
  std::vector<uint64_t> items;
  rk_status st = plan_build_host(S->ctx, inst.data(), (uint32_t)inst.size(), S->cfg.mode, true, &sl.plan, blob, descs,
                                 items);
  uint64_t bb = 0, db = 0, ib = 0;
  if (st == RK_OK) {
    plan_sizes(blob, descs, items, &bb, &db, &ib);
    const bool regrow = bb + db + ib > sl.dplan_cap;
    hipError_t e = ensure_dev(&sl.dplan, &sl.dplan_cap, bb + db + ib);
    if (e == hipSuccess) e = ensure_pinned(&sl.hstage, &sl.hstage_cap, bb + db + ib);
    if (regrow) drop_graphs(sl);  // captured addresses changed
    if (e != hipSuccess) st = alloc_err(S->ctx, e, "step plan buffers");
  }
  // Staging records per tile, from the expected hits per tile (a tile with
  // more is rescanned by the collect pass, a whole extra scan for the dense
  // outputs of merged steps): four times the expected count, between the
  // default (tile bytes / 16) and half the tile, with the slabs of a step
  // kept under 2 GiB.
  sl.slab_cap = 0;
  if (st == RK_OK && S->hits_per_pattern > 0 && nbytes > 0) {
    const uint64_t W = (uint64_t)kTileCfgs[sl.plan.cfg].wg * kTileCfgs[sl.plan.cfg].c;
    // tiles of the step: every image (m-bucket of the merged patterns) scans
    // the corpus once
    const uint64_t tiles = std::max<uint64_t>(1, sl.plan.total_tiles);
    const double per_tile = S->hits_per_pattern * (double)kt / (double)tiles;
    const uint64_t lo = W / 16, hi = std::min<uint64_t>(W / 2, (2ull << 30) / (8 * tiles));
    const uint64_t want = aup((uint64_t)(4.0 * per_tile) + 1, 64);
    if (want > lo && hi > lo) sl.slab_cap = (uint32_t)std::min(want, hi);
  }
  S->ctx->slab_cap = sl.slab_cap;
  Layout L;
  if (st == RK_OK) st = make_layout(S->ctx, &sl.plan, 0, L);
  if (st == RK_OK) {
    const bool regrow = L.total > sl.scratch_cap;
    hipError_t e = ensure_dev(&sl.scratch, &sl.scratch_cap, L.total);
    if (regrow) drop_graphs(sl);
    if (e != hipSuccess) st = alloc_err(S->ctx, e, "step scratch");
  }
  if (st == RK_OK) {
    memset(sl.hstage, 0, bb + db + ib);
    memcpy(sl.hstage, blob.data(), blob.size());
    if (!descs.empty()) memcpy(sl.hstage + bb, descs.data(), descs.size() * sizeof(InstDesc));
    if (!items.empty()) memcpy(sl.hstage + bb + db, items.data(), items.size() * 8);
    sl.plan.dev = nullptr;  // the slot owns the device memory
    sl.plan.blob_dev = (uint8_t *)sl.dplan;
    sl.plan.inst_dev = descs.empty() ? nullptr : (InstDesc *)((uint8_t *)sl.dplan + bb);
    sl.plan.items_dev = items.empty() ? nullptr : (uint64_t *)((uint8_t *)sl.dplan + bb + db);
    sl.plan_bytes = bb + db + ib;
    sl.n_total = nbytes;
    st = run_maybe_graph(S, sl, &sl.gcount, [&]() -> rk_status {
      hipError_t e = hipMemcpyAsync(sl.dplan, sl.hstage, sl.plan_bytes, hipMemcpyHostToDevice, sl.stream);
      if (e != hipSuccess) return hip_err(S->ctx, e, "plan upload");
      rk_status s2 = count_enqueue(S->ctx, &sl.plan, nullptr, 0, sl.scratch, sl.scratch_cap, nullptr, sl.stream);
      if (s2 != RK_OK) return s2;
      e = hipMemcpyAsync(sl.hctr, sl.scratch, 64, hipMemcpyDeviceToHost, sl.stream);
      return e == hipSuccess ? RK_OK : hip_err(S->ctx, e, "count readback");
    });
  }
  if (st == RK_OK) {
    hipError_t e = hipEventRecord(sl.ev_count, sl.stream);
    if (e != hipSuccess) st = hip_err(S->ctx, e, "event");
  }
  lk.lock();
  if (st == RK_ENOMEM && take.size() > 1) {
    // not enough memory for a step this large: its requests go back to the
    // front of the queue and later steps take half as many
    for (auto it = take.rbegin(); it != take.rend(); ++it) S->pending.push_front(*it);
    S->step_limit = (uint32_t)std::max<size_t>(1, take.size() / 2);
    ++S->step_splits;
    return st;
  }
  if (st != RK_OK) {
    for (Request *r : take) finish_request(S, r, st);
    S->cv_done.notify_all();
    return st;
  }
  sl.reqs = take;
  sl.estimated = false;
  sl.step_id = step_id;
  sl.state = kCounting;
  sl.t_start = t0;
  if (S->inflight++ == 0) S->busy_since = now_s();
  ++S->steps;
  S->bytes_scanned += nbytes;
  S->merged_patterns += kt;
  return RK_OK;
}

static void release_slot(rk_server *S, Slot &sl) {
  sl.state = kIdle;
  if (--S->inflight == 0) S->busy_s += now_s() - S->busy_since;
  S->cv_done.notify_all();
}

static void fail_step(rk_server *S, Slot &sl, rk_status st) {
  for (Request *r : sl.reqs) finish_request(S, r, st);
  sl.reqs.clear();
  if (sl.pos_size) S->arena.release(sl.pos_off, sl.pos_size);
  if (sl.aux_size) S->arena.release(sl.aux_off, sl.aux_size);
  sl.pos_size = sl.aux_size = 0;
  release_slot(S, sl);
}

// Admission and collect of a counted step (mu held).  Returns false if the
// arena cannot hold it yet.  The step needs room for its merged positions
// (kept until its requests are released) and for the per-pattern offsets and
// the sort work (until the collect is done).  A step of several requests
// larger than an equal share of the arena per slot is split: its requests go
// back to the front of the queue and later steps take fewer requests.  A
// single request larger than the whole arena fails with RK_ENOSPACE.
static bool try_collect(rk_server *S, Slot &sl, std::unique_lock<std::mutex> &lk) {
  const uint32_t k = sl.plan.k_total;
  const uint64_t pos_b = aup(std::max<uint64_t>(sl.total, 1) * 8, 256);
  const uint64_t off_b = aup((uint64_t)(k + 1) * 8, 256);
  const uint64_t work_b = aup(work_bytes_for(&sl.plan, sl.total), 256);
  const uint64_t need = pos_b + off_b + work_b;
  const uint64_t share = S->arena.cap / S->slots.size();
  if (k && !sl.estimated) {
    sl.estimated = true;
    const double hpp = (double)sl.total / (double)k;
    S->hits_per_pattern = S->hits_per_pattern < 0 ? hpp : 0.7 * S->hits_per_pattern + 0.3 * hpp;
  }
  rk_status st = RK_OK;
  if (sl.reqs.size() > 1 && need > share) {
    const uint64_t parts = std::max<uint64_t>(2, (need + share - 1) / std::max<uint64_t>(share, 1));
    S->step_limit = (uint32_t)std::max<uint64_t>(1, sl.reqs.size() / parts);
    for (auto it = sl.reqs.rbegin(); it != sl.reqs.rend(); ++it) S->pending.push_front(*it);
    sl.reqs.clear();
    ++S->step_splits;
    release_slot(S, sl);
    return true;
  }
  if (need > S->arena.cap) {
    st = set_err(S->ctx, RK_ENOSPACE, "request needs %llu arena bytes (arena %llu)", (unsigned long long)need,
                 (unsigned long long)S->arena.cap);
  } else {
    uint64_t poff, aoff;
    if (!S->arena.alloc(pos_b, &poff)) return false;
    if (!S->arena.alloc(off_b + work_b, &aoff)) {
      S->arena.release(poff, pos_b);
      return false;
    }
    sl.pos_off = poff;
    sl.pos_size = pos_b;
    sl.aux_off = aoff;
    sl.aux_size = off_b + work_b;
    // steps that use little of the arena let later steps take more requests
    if (need * 4 <= share && S->step_limit < S->cfg.max_step_requests)
      S->step_limit = (uint32_t)std::min<uint64_t>((uint64_t)S->step_limit * 2, S->cfg.max_step_requests);
    lk.unlock();
    uint8_t *aux = (uint8_t *)S->arena_dev + aoff;
    uint64_t *doff = (uint64_t *)aux, *dpos = (uint64_t *)((uint8_t *)S->arena_dev + poff);
    void *work = work_b ? aux + off_b : nullptr;
    hipError_t e = ensure_pinned(&sl.hres, &sl.hres_cap, (uint64_t)(k + 1) * 8);
    if (e != hipSuccess) st = hip_err(S->ctx, e, "offset staging");
    if (st == RK_OK)
      st = run_maybe_graph(S, sl, &sl.gcollect, [&]() -> rk_status {
        S->ctx->slab_cap = sl.slab_cap;  // the layout of this step's count pass
        rk_status s2 = collect_enqueue_known(S->ctx, &sl.plan, nullptr, 0, sl.scratch, sl.scratch_cap, work, work_b,
                                             doff, dpos, std::max<uint64_t>(sl.total, 1), sl.total, sl.ovf,
                                             sl.stream);
        if (s2 != RK_OK) return s2;
        hipError_t e2 = hipMemcpyAsync(sl.hres, doff, (uint64_t)(k + 1) * 8, hipMemcpyDeviceToHost, sl.stream);
        return e2 == hipSuccess ? RK_OK : hip_err(S->ctx, e2, "offset copy");
      });
    if (st == RK_OK) {
      e = hipEventRecord(sl.ev_collect, sl.stream);
      if (e != hipSuccess) st = hip_err(S->ctx, e, "event");
    }
    lk.lock();
    if (st == RK_OK) {
      sl.state = kCollecting;
      return true;
    }
  }
  fail_step(S, sl, st);
  return true;
}

// Collected step: every request gets its slice of the merged positions and
// its own offsets; the per-pattern offsets and the sort work go back to the
// arena (mu held).
static void finish_collect(rk_server *S, Slot &sl) {
  StepBuf *buf = new (std::nothrow) StepBuf();
  if (!buf) {
    fail_step(S, sl, set_err(S->ctx, RK_ENOMEM, "step buffer"));
    return;
  }
  buf->off = sl.pos_off;
  buf->size = sl.pos_size;
  buf->refs = (uint32_t)sl.reqs.size();
  const uint64_t *off = sl.hres;
  for (Request *r : sl.reqs) {
    const uint64_t b = off[r->gp0];
    r->res_offsets.resize(r->k + 1);
    for (uint32_t j = 0; j <= r->k; ++j) r->res_offsets[j] = off[r->gp0 + j] - b;
    r->out_off = sl.pos_off + b * 8;
    r->out_size = r->res_offsets[r->k] * 8;
    r->buf = buf;
    r->bytes.clear();
    r->bytes.shrink_to_fit();
    finish_request(S, r, RK_OK);
  }
  if (sl.reqs.empty()) {
    S->arena.release(buf->off, buf->size);
    delete buf;
  }
  sl.reqs.clear();
  S->arena.release(sl.aux_off, sl.aux_size);
  sl.pos_size = sl.aux_size = 0;  // the positions now belong to the requests
  release_slot(S, sl);
}

static void scheduler(rk_server *S) {
  hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  while (true) {
    bool progress = false;
    for (Slot &sl : S->slots) {
      if (sl.state == kCounting) {
        const hipError_t q = hipEventQuery(sl.ev_count);
        if (q == hipSuccess) {
          sl.total = sl.hctr[0];
          sl.ovf = ovf_total(sl.hctr);
          sl.state = kCounted;
          progress = true;
        } else if (q != hipErrorNotReady) {
          fail_step(S, sl, hip_err(S->ctx, q, "count pass"));
        }
      }
      if (sl.state == kCounted) {
        if (try_collect(S, sl, lk)) {
          sl.wait_since = 0;
          progress = true;
        } else {
          // No room in the arena.  Steps in flight free their sort work when
          // their collect ends; with none in flight only the client's
          // releases can make room, so the wait is bounded.
          bool others = false;
          for (Slot &o : S->slots) others |= &o != &sl && (o.state == kCounting || o.state == kCollecting);
          const double t = now_s();
          if (sl.wait_since == 0) ++S->admission_waits;
          if (others || sl.wait_since == 0) {
            sl.wait_since = t;
          } else if (t - sl.wait_since > S->cfg.admission_timeout_s) {
            fail_step(S, sl, set_err(S->ctx, RK_ENOSPACE,
                                     "no arena space for a step of %llu hits for %.3f s with no step in flight: "
                                     "unreleased results hold %llu of %llu bytes",
                                     (unsigned long long)sl.total, S->cfg.admission_timeout_s,
                                     (unsigned long long)S->arena.used, (unsigned long long)S->arena.cap));
            sl.wait_since = 0;
            S->cv_done.notify_all();
            progress = true;
          }
        }
      }
      if (sl.state == kCollecting) {
        const hipError_t q = hipEventQuery(sl.ev_collect);
        if (q == hipSuccess) {
          finish_collect(S, sl);
          progress = true;
        } else if (q != hipErrorNotReady) {
          fail_step(S, sl, hip_err(S->ctx, q, "collect pass"));
        }
      }
    }
    if (S->stop && S->inflight == 0) break;
    if (S->cfg.request_timeout_s > 0 && !S->pending.empty()) {
      // requests that waited too long for a step (the oldest are in front)
      const double t = now_s();
      bool any = false;
      while (!S->pending.empty() && t - S->pending.front()->t_submit > S->cfg.request_timeout_s) {
        finish_request(S, S->pending.front(), RK_ETIMEDOUT);
        S->pending.pop_front();
        any = true;
      }
      if (any) S->cv_done.notify_all();
    }
    if (!S->stop) {
      for (Slot &sl : S->slots) {
        if (sl.state != kIdle || S->pending.empty()) continue;
        // a slot whose counted step waits for memory keeps later steps out,
        // so that admission stays in arrival order
        bool waiting = false;
        for (Slot &o : S->slots) waiting |= o.state == kCounted;
        if (waiting) break;
        start_step(S, sl, lk);
        progress = true;
      }
    }
    if (progress) continue;
    if (S->inflight) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    } else {
      S->cv_submit.wait_for(lk, std::chrono::milliseconds(20));
    }
  }
}

}  // namespace rk

extern "C" {

void rk_server_cfg_default(rk_server_cfg *cfg) {
  if (!cfg) return;
  cfg->arena_bytes = 4ull << 30;
  cfg->max_inflight = 2;
  cfg->max_step_requests = 4096;
  cfg->max_step_patterns = 1024;
  cfg->mode = RK_MODE_SCREEN;
  cfg->use_graphs = 1;
  cfg->admission_timeout_s = 2.0;
  cfg->request_timeout_s = 0.0;
}

rk_status rk_server_create(rk_ctx *ctx, const rk_server_cfg *cfg_in, rk_server **out) {
  if (!ctx || !out) return RK_EINVAL;
  *out = nullptr;
  rk_server_cfg cfg;
  rk_server_cfg_default(&cfg);
  if (cfg_in) cfg = *cfg_in;
  if (cfg.max_inflight < 1 || cfg.max_inflight > 8) return set_err(ctx, RK_EINVAL, "max_inflight must be 1..8");
  if (cfg.max_step_requests < 1 || cfg.max_step_patterns < 1) return set_err(ctx, RK_EINVAL, "step limits must be >= 1");
  if (cfg.mode == RK_MODE_AUTO) cfg.mode = RK_MODE_SCREEN;
  if (cfg.mode != RK_MODE_SCREEN && cfg.mode != RK_MODE_EXACT) return set_err(ctx, RK_EINVAL, "unknown mode");
  if (!(cfg.admission_timeout_s >= 0) || !(cfg.request_timeout_s >= 0))
    return set_err(ctx, RK_EINVAL, "timeouts must be >= 0");
  rk_server *S = new (std::nothrow) rk_server();
  if (!S) return RK_ENOMEM;
  S->cfg = cfg;
  S->device = ctx->device;
  rk_status st = rk_ctx_create(ctx->device, 256, kQ, &S->ctx);
  if (st != RK_OK) {
    delete S;
    return set_err(ctx, st, "server context");
  }
  // fixed persistent grid: no occupancy query while a stream is being captured
  S->ctx->grid = (uint32_t)S->ctx->num_cu * 4;
  // staging records per tile: the plan default (one per 16 text bytes for
  // pattern sets), since served requests are hit-dense and a tile whose
  // records overflow is scanned a second time
  for (int md = 0; md < 3; ++md)
    for (int m = 0; m <= RK_MAX_M; ++m) S->ctx->tune[md][m] = ctx->tune[md][m];
  S->ctx->tile_cfg = ctx->tile_cfg;
  hipError_t e = hipMalloc(&S->arena_dev, std::max<uint64_t>(cfg.arena_bytes, 4096));
  if (e != hipSuccess) {
    rk_ctx_destroy(S->ctx);
    delete S;
    return set_err(ctx, RK_ENOMEM, "server arena (%llu bytes)", (unsigned long long)cfg.arena_bytes);
  }
  S->arena.init(cfg.arena_bytes);
  S->step_limit = cfg.max_step_requests;
  S->slots.resize(cfg.max_inflight);
  e = hipStreamCreateWithFlags(&S->fetch_stream, hipStreamNonBlocking);
  for (Slot &sl : S->slots) {
    if (e != hipSuccess) break;
    e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev_count, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev_collect, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void **)&sl.hctr, 64, hipHostMallocDefault);
    if (e != hipSuccess) break;
  }
  if (e != hipSuccess) {
    rk_server_destroy(S);
    return set_err(ctx, RK_EDEVICE, "server streams: %s", hipGetErrorString(e));
  }
  try {
    S->th = std::thread(scheduler, S);
  } catch (...) {
    rk_server_destroy(S);
    return set_err(ctx, RK_ENOMEM, "scheduler thread");
  }
  *out = S;
  return RK_OK;
}

rk_status rk_server_add_corpus(rk_server *S, const uint8_t *text, uint64_t n, uint32_t *id) {
  if (!S || !id || (n && !text)) return RK_EINVAL;
  if (((uintptr_t)text & 15u) != 0) return RK_EINVAL;
  if (n > RK_MAX_N) return RK_EUNSUPPORTED;
  std::lock_guard<std::mutex> g(S->mu);
  S->corpora.push_back({text, n});
  *id = (uint32_t)(S->corpora.size() - 1);
  return RK_OK;
}

rk_status rk_server_submit(rk_server *S, uint32_t corpus, const uint8_t *bytes, const uint64_t *offs, uint32_t k,
                           uint64_t *req_id) {
  if (!S || !req_id || (k && !offs)) return RK_EINVAL;
  for (uint32_t j = 0; j < k; ++j) {
    if (offs[j + 1] <= offs[j]) return RK_EINVAL;
    if (offs[j + 1] - offs[j] > RK_MAX_M) return RK_EUNSUPPORTED;
  }
  if (k && !bytes && offs[k] > offs[0]) return RK_EINVAL;
  Request *r = new (std::nothrow) Request();
  if (!r) return RK_ENOMEM;
  r->corpus = corpus;
  r->k = k;
  if (k) {
    r->bytes.assign(bytes + offs[0], bytes + offs[k]);
    r->offs.resize(k + 1);
    for (uint32_t j = 0; j <= k; ++j) r->offs[j] = offs[j] - offs[0];
  }
  r->t_submit = now_s();
  std::lock_guard<std::mutex> g(S->mu);
  if (corpus >= S->corpora.size()) {
    delete r;
    return RK_EINVAL;
  }
  r->id = S->next_id++;
  S->reqs[r->id] = r;
  ++S->submitted;
  ++S->outstanding;
  *req_id = r->id;
  if (k == 0) {
    r->res_offsets.assign(1, 0);
    finish_request(S, r, RK_OK);
    S->cv_done.notify_all();
    return RK_OK;
  }
  S->pending.push_back(r);
  S->cv_submit.notify_one();
  return RK_OK;
}

static void fill_view(const rk_server *S, const Request *r, rk_result_view *out) {
  out->status = r->status;
  out->k = r->k;
  out->offsets = r->res_offsets.empty() ? nullptr : r->res_offsets.data();
  out->positions_dev = (r->status == RK_OK && r->out_size) ? (const uint64_t *)((uint8_t *)S->arena_dev + r->out_off)
                                                           : nullptr;
  out->t_submit = r->t_submit;
  out->t_start = r->t_start;
  out->t_done = r->t_done;
  out->step = r->step;
}

rk_status rk_server_poll(rk_server *S, uint64_t id, rk_result_view *out) {
  if (!S || !out) return RK_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return RK_EINVAL;
  fill_view(S, it->second, out);
  return it->second->status == RK_EBUSY ? RK_EBUSY : RK_OK;
}

rk_status rk_server_wait(rk_server *S, uint64_t id, double timeout_s, rk_result_view *out) {
  if (!S || !out) return RK_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return RK_EINVAL;
  Request *r = it->second;
  const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
  while (r->status == RK_EBUSY)
    if (S->cv_done.wait_until(lk, until) == std::cv_status::timeout && r->status == RK_EBUSY) break;
  fill_view(S, r, out);
  return r->status == RK_EBUSY ? RK_EBUSY : RK_OK;
}

rk_status rk_server_cancel(rk_server *S, uint64_t id) {
  if (!S) return RK_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return RK_EINVAL;
  Request *r = it->second;
  auto p = std::find(S->pending.begin(), S->pending.end(), r);
  if (p == S->pending.end()) return r->status == RK_EBUSY ? RK_EBUSY : RK_OK;
  S->pending.erase(p);
  finish_request(S, r, RK_ECANCELED);
  S->cv_done.notify_all();
  return RK_OK;
}

rk_status rk_server_release(rk_server *S, uint64_t id) {
  if (!S) return RK_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  auto it = S->reqs.find(id);
  if (it == S->reqs.end()) return RK_EINVAL;
  if (it->second->status == RK_EBUSY) return RK_EBUSY;
  Request *r = it->second;
  if (r->buf && --r->buf->refs == 0) {
    S->arena.release(r->buf->off, r->buf->size);
    delete r->buf;
  }
  delete r;
  S->reqs.erase(it);
  // ids released before rk_server_next_done reported them are dropped from
  // the completion queue once they outnumber the live requests
  if (S->done_q.size() > 2 * S->reqs.size() + 1024) {
    std::deque<uint64_t> keep;
    for (uint64_t d : S->done_q)
      if (S->reqs.count(d)) keep.push_back(d);
    S->done_q.swap(keep);
  }
  return RK_OK;
}

rk_status rk_server_next_done(rk_server *S, double timeout_s, uint64_t *req_id) {
  if (!S || !req_id) return RK_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
  for (;;) {
    while (!S->done_q.empty()) {
      const uint64_t id = S->done_q.front();
      S->done_q.pop_front();
      if (S->reqs.count(id)) {
        *req_id = id;
        return RK_OK;
      }
    }
    if (S->cv_done.wait_until(lk, until) == std::cv_status::timeout && S->done_q.empty()) return RK_EBUSY;
  }
}

rk_status rk_server_fetch(rk_server *S, uint64_t id, uint64_t *positions_host, uint64_t cap) {
  if (!S) return RK_EINVAL;
  uint64_t off = 0, bytes = 0;
  {
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(id);
    if (it == S->reqs.end()) return RK_EINVAL;
    const Request *r = it->second;
    if (r->status == RK_EBUSY) return RK_EBUSY;
    if (r->status != RK_OK) return r->status;
    off = r->out_off;
    bytes = r->out_size;
  }
  if (bytes / 8 > cap) return RK_ENOSPACE;
  if (bytes && !positions_host) return RK_EINVAL;
  if (!bytes) return RK_OK;
  hipSetDevice(S->device);
  // the slice stays allocated until rk_server_release (the caller's); the copy
  // runs on the server's own non-blocking stream, so that it neither waits for
  // nor conflicts with steps being captured or run on the slot streams
  hipError_t e = hipMemcpyAsync(positions_host, (uint8_t *)S->arena_dev + off, bytes, hipMemcpyDeviceToHost,
                                S->fetch_stream);
  if (e == hipSuccess) e = hipStreamSynchronize(S->fetch_stream);
  return e == hipSuccess ? RK_OK : RK_EDEVICE;
}

rk_status rk_server_drain(rk_server *S) {
  if (!S) return RK_EINVAL;
  std::unique_lock<std::mutex> lk(S->mu);
  while (S->outstanding) S->cv_done.wait_for(lk, std::chrono::milliseconds(50));
  return RK_OK;
}

rk_status rk_server_get_stats(rk_server *S, rk_server_stats *o) {
  if (!S || !o) return RK_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  memset(o, 0, sizeof *o);
  o->submitted = S->submitted;
  o->completed = S->completed;
  o->canceled = S->canceled;
  o->failed = S->failed;
  o->steps = S->steps;
  o->bytes_scanned = S->bytes_scanned;
  o->merged_patterns = S->merged_patterns;
  o->request_patterns = S->request_patterns;
  o->busy_s = S->busy_s + (S->inflight ? now_s() - S->busy_since : 0.0);
  o->arena_high_water = S->arena.high;
  o->queue_depth = (uint32_t)S->pending.size();
  o->inflight = S->inflight;
  o->admission_waits = S->admission_waits;
  o->step_splits = S->step_splits;
  if (!S->lat_ms.empty()) {
    std::vector<double> v = S->lat_ms;
    std::sort(v.begin(), v.end());
    auto q = [&v](double f) { return v[std::min(v.size() - 1, (size_t)(f * (v.size() - 1) + 0.5))]; };
    o->p50_ms = q(0.50);
    o->p99_ms = q(0.99);
    o->max_ms = v.back();
    double s = 0;
    for (double x : v) s += x;
    o->mean_ms = s / v.size();
  }
  return RK_OK;
}

rk_status rk_server_reset_stats(rk_server *S) {
  if (!S) return RK_EINVAL;
  std::lock_guard<std::mutex> g(S->mu);
  S->lat_ms.clear();
  S->completed = S->canceled = S->failed = S->steps = S->bytes_scanned = 0;
  S->merged_patterns = S->request_patterns = S->admission_waits = S->step_splits = 0;
  S->submitted = S->outstanding;
  S->busy_s = 0;
  if (S->inflight) S->busy_since = now_s();
  S->arena.high = S->arena.used;
  return RK_OK;
}

void rk_server_destroy(rk_server *S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> g(S->mu);
    S->stop = true;
    for (Request *r : S->pending) finish_request(S, r, RK_ECANCELED);
    S->pending.clear();
    S->cv_submit.notify_all();
    S->cv_done.notify_all();
  }
  if (S->th.joinable()) S->th.join();
  hipSetDevice(S->device);
  for (Slot &sl : S->slots) {
    if (sl.stream) hipStreamSynchronize(sl.stream);
    drop_graphs(sl);
    if (sl.ev_count) hipEventDestroy(sl.ev_count);
    if (sl.ev_collect) hipEventDestroy(sl.ev_collect);
    if (sl.stream) hipStreamDestroy(sl.stream);
    if (sl.dplan) hipFree(sl.dplan);
    if (sl.scratch) hipFree(sl.scratch);
    if (sl.hstage) hipHostFree(sl.hstage);
    if (sl.hres) hipHostFree(sl.hres);
    if (sl.hctr) hipHostFree(sl.hctr);
  }
  if (S->fetch_stream) hipStreamDestroy(S->fetch_stream);
  if (S->arena_dev) hipFree(S->arena_dev);
  for (auto &kv : S->reqs) {
    Request *r = kv.second;
    if (r->buf && --r->buf->refs == 0) delete r->buf;
    delete r;
  }
  if (S->ctx) rk_ctx_destroy(S->ctx);
  delete S;
}

}  // extern "C"
