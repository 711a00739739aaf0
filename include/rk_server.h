/*
 * rk_server.h -- continuous-batching search server of librk.
 *
 * Corpora stay resident in device memory.  Clients submit searches (a corpus
 * id and a pattern set, the problem of Sec. 1 of Shah & Oza: every occurrence
 * of every pattern) from any thread.  A scheduler thread forms steps from the
 * requests that are waiting: a step serves the corpus of the oldest waiting
 * request together with every other waiting request for that corpus (up to
 * the step limits and an output estimate), concatenating their patterns
 * (identical patterns share their bytes in the table image), so that they
 * share one scan (the batch path of rk.h).  Each
 * step runs count -> admission -> collect: the count pass gives the exact
 * output size, the step is admitted when the output arena can hold it (a
 * step too large for its share of the arena goes back to the queue and is
 * split), and collect writes every hit sorted by merged pattern id, so that
 * each request's result is a contiguous slice of the step's output without a
 * copy (results stay in device memory until the client releases them; the
 * host gets per-pattern offsets, and positions on demand).
 * Several steps are in flight at once on separate streams, so requests that
 * arrive while others run on the device are admitted as slots and arena space
 * free up.  With use_graphs, the count and the collect pass of a step are each
 * captured into a graph that updates the slot's executable graph in place
 * (re-instantiated only when the launch sequence changes) and launched as one
 * unit.  A step that fails for lack of memory before it reaches the device
 * (host or device allocations of its plan) goes back to the queue and later
 * steps take fewer requests; a single request that fails that way, and every
 * step that fails on the device, end with the error.
 *
 * Results are exact and identical to a solo rk_count/rk_collect of the same
 * request: merging only changes which patterns share a scan.
 *
 * While the server captures a step, work that a client enqueues on the
 * legacy default stream of the same device may be refused by the runtime
 * (the legacy stream would wait on a capturing stream): clients that work on
 * the device beside a running server use streams of their own (the library's
 * own uploads, rk_plan_create included, never use the legacy stream).
 */
#ifndef RK_SERVER_H
#define RK_SERVER_H

#include "rk.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rk_server rk_server;

typedef struct {
  uint64_t arena_bytes;        /* device memory for hits of steps in flight and of finished,
                                  unreleased requests (default 4 GiB).  A counted step waits
                                  until the arena can hold it, so results must be released
                                  as they are consumed.  Requests complete out of submission
                                  order (a later request for the oldest request's corpus joins
                                  its step): a client that releases only in submission order,
                                  or waits for every request before releasing any, can hold
                                  the arena full; such a step ends RK_ENOSPACE after
                                  admission_timeout_s. */
  uint32_t max_inflight;       /* steps in flight on the device, 1..8 (default 2) */
  uint32_t max_step_requests;  /* requests merged into one step (default 4096) */
  uint32_t max_step_patterns;  /* merged patterns per step (default 1024; a request with
                                  more still forms a step of its own).  Larger steps share
                                  one scan among more requests but cost more per hit (larger
                                  tables, more candidates per tile, wider sort keys): on the
                                  64-corpus Zipf-text workload overloaded at 2,000 req/s,
                                  steps of 256 / 512 / 1,024 / 2,048 / 262,144 merged
                                  patterns served 458 / 663 / 808 / 563 / 305 req/s. */
  int mode;                    /* rk_mode of every search */
  int use_graphs;              /* 1: launch each step's passes as HIP graphs (captured per step into the
                                  slot's executable graph, updated in place); 0: plain launches */
  double admission_timeout_s;  /* a counted step that finds no arena space while no other step is in
                                  flight (only unreleased results hold the arena) waits at most this
                                  long for the client to release some, then its requests end
                                  RK_ENOSPACE (default 2 s; a step never waits forever) */
  double request_timeout_s;    /* a request still waiting for a step after this long ends
                                  RK_ETIMEDOUT (0, the default: no limit) */
} rk_server_cfg;

/* Fills cfg with the defaults above. */
void rk_server_cfg_default(rk_server_cfg *cfg);

typedef struct {
  rk_status status;            /* RK_OK done, RK_EBUSY pending, RK_ECANCELED, RK_ETIMEDOUT, RK_ENOSPACE
                                  (admission timed out), or the step's error */
  uint32_t k;                  /* patterns of the request */
  const uint64_t *offsets;     /* host, k+1 entries; valid until rk_server_release */
  const uint64_t *positions_dev; /* device (server arena), offsets[k] entries, per pattern
                                    ascending; valid until rk_server_release */
  double t_submit, t_start, t_done; /* seconds on the server's monotonic clock */
  uint64_t step;               /* step that served the request */
} rk_result_view;

typedef struct {
  uint64_t submitted, completed, canceled, failed;
  uint64_t steps;
  uint64_t bytes_scanned;      /* corpus bytes scanned by all steps */
  uint64_t merged_patterns;    /* patterns searched after merging, over all steps */
  uint64_t request_patterns;   /* patterns submitted, over all completed requests */
  double p50_ms, p99_ms, mean_ms, max_ms; /* submit -> done latency of completed requests */
  double busy_s;               /* wall time with at least one step in flight */
  uint64_t arena_high_water;   /* bytes */
  uint32_t queue_depth;        /* requests waiting for a step */
  uint32_t inflight;           /* steps on the device */
  uint64_t admission_waits;    /* counted steps that waited for arena space */
  uint64_t step_splits;        /* counted steps given back to the queue as too large */
} rk_server_stats;

/* Creates a server on ctx's device (batches of Sec. 1's problem on resident
 * texts; the paper runs one search per launch, Sec. 3.1).  The server owns its streams, graphs,
 * arena and scheduler thread; ctx must outlive it and is not used by the
 * server's thread (the server keeps its own context on the same device). */
rk_status rk_server_create(rk_ctx *ctx, const rk_server_cfg *cfg, rk_server **out);
/* Registers a resident corpus (device memory, 16-byte aligned, caller-owned,
 * unchanged while the server runs).  Thread-safe. */
rk_status rk_server_add_corpus(rk_server *srv, const uint8_t *text_dev, uint64_t n, uint32_t *corpus_id);
/* Queues a search of corpus_id for k patterns (host arrays, copied): every
 * occurrence of every pattern, as rk_count + rk_collect would give (Sec. 1).
 * Thread-safe.  Pattern lengths as in rk.h. */
rk_status rk_server_submit(rk_server *srv, uint32_t corpus_id, const uint8_t *bytes_host,
                           const uint64_t *offsets_host, uint32_t k, uint64_t *req_id);
/* Non-blocking: RK_EBUSY while the request is pending, else fills out. */
rk_status rk_server_poll(rk_server *srv, uint64_t req_id, rk_result_view *out);
/* Blocks until the request is done or timeout_s passes (RK_EBUSY). */
rk_status rk_server_wait(rk_server *srv, uint64_t req_id, double timeout_s, rk_result_view *out);
/* Blocks until a request has finished that no earlier call returned, and
 * gives its id: requests are reported once each, in the order they finished
 * (done, canceled or failed), so a client can consume results as they come
 * and release them at once.  RK_EBUSY if none finishes within timeout_s.  A
 * request released before it was reported is skipped. */
rk_status rk_server_next_done(rk_server *srv, double timeout_s, uint64_t *req_id);
/* Cancels a request that has not been put into a step (RK_EBUSY otherwise). */
rk_status rk_server_cancel(rk_server *srv, uint64_t req_id);
/* Copies a finished request's positions (offsets[k] entries) to host memory;
 * cap = entries available at positions_host.  Synchronous. */
rk_status rk_server_fetch(rk_server *srv, uint64_t req_id, uint64_t *positions_host, uint64_t cap);
/* Frees a finished request's results.  Its positions are a slice of its
 * step's output block, which returns to the arena once every request of the
 * step has been released. */
rk_status rk_server_release(rk_server *srv, uint64_t req_id);
/* Blocks until every submitted request is finished. */
rk_status rk_server_drain(rk_server *srv);
rk_status rk_server_get_stats(rk_server *srv, rk_server_stats *out);
/* Clears the latency record and counters (corpora and requests stay). */
rk_status rk_server_reset_stats(rk_server *srv);
/* Stops the scheduler (pending requests end RK_ECANCELED) and frees everything. */
void rk_server_destroy(rk_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* RK_SERVER_H */
