/*
 * Reference oracle for multi-pattern Rabin-Karp search.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP implementation.
 *
 * What it computes (Shah & Oza, "Improved Parallel Rabin-Karp Algorithm Using
 * CUDA", Sec. 3.1 and its sequential pseudo code):
 *   - the pattern hash hx and the window hash hy are the polynomial
 *         h(s[0..m)) = sum_{i<m} s[i] * d^(m-1-i)   (mod q)
 *     evaluated by Horner's rule h <- h*d + s[i]  (the paper's shift-and-add
 *     form is the case d = 2 with no explicit modulus; this oracle takes the
 *     base d and the modulus q as parameters, defaulting to d = 256,
 *     q = 2^61 - 1);
 *   - a window x is reported for pattern P iff hy(x) == hx and the bytes
 *     compare equal (Sec. 3.1: bytes are compared only after the hashes agree);
 *   - windows run over every x in [0, n-m] inclusive (the GPU pseudo code's
 *     guard x <= n-m; the sequential loop bound x < n-m would drop the last
 *     window, which is read as a slip);
 *   - several patterns are searched at once (the paper's stated focus on
 *     multiple-pattern matching, Sec. 1): every pattern gets its own ascending
 *     list of positions; duplicated patterns each get the full list.
 *
 * Arithmetic: every product and sum is formed in unsigned __int128 and reduced
 * with the % operator, so no lazy reduction or modulus-specific trick is used.
 * Bytes are unsigned (0..255).
 *
 * Functions:
 *   rko_hash            Horner evaluation of one string            (Sec. 3.1)
 *   rko_pow             d^e mod q by repeated squaring (textbook)
 *   rko_window_hashes   hy for chosen windows, each by direct Horner (Sec. 3.1)
 *   rko_search_recompute  the paper's loop as written: hy recomputed per window
 *   rko_search          textbook rolling Rabin-Karp over every window,
 *                       multi-pattern, optional thread split of the windows
 *   rko_brute           the definition: byte comparison at every window
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

#define RKO_OK 0
#define RKO_EINVAL -1
#define RKO_ENOMEM -2

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t q) {
  return (uint64_t)(((u128)a * (u128)b) % (u128)q);
}

static uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) {
  return (uint64_t)(((u128)a + (u128)b) % (u128)q);
}

/* Horner: h <- h*d + s[i] (mod q), i = 0..m-1. */
uint64_t rko_hash(const uint8_t *s, uint64_t m, uint64_t d, uint64_t q) {
  uint64_t h = 0;
  for (uint64_t i = 0; i < m; ++i) h = addmod(mulmod(h, d, q), (uint64_t)s[i] % q, q);
  return h;
}

uint64_t rko_pow(uint64_t d, uint64_t e, uint64_t q) {
  uint64_t r = 1 % q, b = d % q;
  while (e) {
    if (e & 1) r = mulmod(r, b, q);
    b = mulmod(b, b, q);
    e >>= 1;
  }
  return r;
}

static int check_params(uint64_t d, uint64_t q) {
  if (q < 2 || q >= (1ull << 63)) return RKO_EINVAL;
  if (d == 0 || d >= q) return RKO_EINVAL;
  return RKO_OK;
}

/* out[i] = hash of text[xs[i] .. xs[i]+m); requires xs[i] + m <= n. */
int rko_window_hashes(const uint8_t *text, uint64_t n, uint64_t m, uint64_t d, uint64_t q,
                      const uint64_t *xs, uint64_t cnt, uint64_t *out) {
  if (check_params(d, q) || m == 0 || m > n) return RKO_EINVAL;
  for (uint64_t i = 0; i < cnt; ++i) {
    if (xs[i] > n - m) return RKO_EINVAL;
    out[i] = rko_hash(text + xs[i], m, d, q);
  }
  return RKO_OK;
}

/* ---- growable list of (pattern id, position) hits, appended in x order ---- */
typedef struct {
  uint32_t *pid;
  uint64_t *pos;
  uint64_t len, cap;
} hitlist;

static int hl_push(hitlist *h, uint32_t pid, uint64_t pos) {
  if (h->len == h->cap) {
    uint64_t nc = h->cap ? 2 * h->cap : 256;
    uint32_t *np_ = (uint32_t *)realloc(h->pid, nc * sizeof(uint32_t));
    if (!np_) return RKO_ENOMEM;
    h->pid = np_;
    uint64_t *nq = (uint64_t *)realloc(h->pos, nc * sizeof(uint64_t));
    if (!nq) return RKO_ENOMEM;
    h->pos = nq;
    h->cap = nc;
  }
  h->pid[h->len] = pid;
  h->pos[h->len] = pos;
  h->len++;
  return RKO_OK;
}

static void hl_free(hitlist *h) {
  free(h->pid);
  free(h->pos);
  h->pid = NULL;
  h->pos = NULL;
  h->len = h->cap = 0;
}

/* ---- pattern set: for each distinct length, the (hash, id) pairs sorted by hash ---- */
typedef struct {
  uint64_t m;
  uint64_t npat;
  uint64_t *hash; /* sorted ascending */
  uint32_t *id;   /* id[i] belongs to hash[i]; equal hashes keep ascending id */
} lengroup;

typedef struct {
  const uint8_t *text;
  uint64_t n;
  const uint8_t *pbytes;
  const uint64_t *poff;
  uint64_t d, q;
  const lengroup *g;
  uint64_t ng;
  int recompute; /* 1: hy recomputed from scratch per window (the paper's loop) */
  uint64_t x_begin, x_end; /* this worker scans windows whose start lies in [x_begin, x_end) */
  hitlist out;
  int status;
} worker;

static int cmp_pair(const void *a, const void *b) {
  const uint64_t *pa = (const uint64_t *)a, *pb = (const uint64_t *)b;
  if (pa[0] != pb[0]) return pa[0] < pb[0] ? -1 : 1;
  if (pa[1] != pb[1]) return pa[1] < pb[1] ? -1 : 1;
  return 0;
}

/* lower bound of h in the sorted hash array */
static uint64_t lower_bound(const uint64_t *a, uint64_t len, uint64_t h) {
  uint64_t lo = 0, hi = len;
  while (lo < hi) {
    uint64_t mid = lo + (hi - lo) / 2;
    if (a[mid] < h) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

/* Report x for every pattern of group g whose hash equals hy and whose bytes match. */
static int probe_and_verify(worker *w, const lengroup *g, uint64_t x, uint64_t hy) {
  uint64_t i = lower_bound(g->hash, g->npat, hy);
  for (; i < g->npat && g->hash[i] == hy; ++i) {
    uint32_t id = g->id[i];
    if (memcmp(w->pbytes + w->poff[id], w->text + x, g->m) == 0) {
      int s = hl_push(&w->out, id, x);
      if (s) return s;
    }
  }
  return RKO_OK;
}

/* One worker: for every length group, every window start in [x_begin, x_end). */
static void *run_worker(void *arg) {
  worker *w = (worker *)arg;
  w->status = RKO_OK;
  /* windows are visited in x order; at one x the groups are visited in
   * length order; the final per-pattern lists only depend on x order. */
  for (uint64_t gi = 0; gi < w->ng; ++gi) {
    const lengroup *g = &w->g[gi];
    uint64_t m = g->m;
    if (m > w->n) continue;
    uint64_t last = w->n - m; /* last valid window start */
    uint64_t xb = w->x_begin, xe = w->x_end;
    if (xe > last + 1) xe = last + 1;
    if (xb >= xe) continue;
    if (w->recompute) {
      for (uint64_t x = xb; x < xe; ++x) {
        uint64_t hy = rko_hash(w->text + x, m, w->d, w->q);
        int s = probe_and_verify(w, g, x, hy);
        if (s) { w->status = s; return NULL; }
      }
    } else {
      /* rolling update:  hy(x+1) = d*hy(x) - T[x]*d^m + T[x+m]   (mod q) */
      uint64_t dm = rko_pow(w->d, m, w->q);
      uint64_t hy = rko_hash(w->text + xb, m, w->d, w->q);
      for (uint64_t x = xb;; ++x) {
        int s = probe_and_verify(w, g, x, hy);
        if (s) { w->status = s; return NULL; }
        if (x + 1 >= xe) break;
        uint64_t out_term = mulmod((uint64_t)w->text[x], dm, w->q);
        uint64_t v = mulmod(hy, w->d, w->q);
        v = addmod(v, w->q - out_term, w->q);
        v = addmod(v, (uint64_t)w->text[x + m], w->q);
        hy = v;
      }
    }
  }
  return NULL;
}

/*
 * Search text[0..n) for k patterns (pattern j = pbytes[poff[j] .. poff[j+1])).
 * On success *offsets_out (k+1 entries) and *positions_out are malloc'd; pattern
 * j's ascending positions are positions[offsets[j] .. offsets[j+1]).  Free both
 * with rko_free.  nthreads >= 1 splits the window range into contiguous parts.
 * recompute != 0 evaluates every window hash from scratch (the paper's loop).
 */
static int search_impl(const uint8_t *text, uint64_t n, const uint8_t *pbytes,
                       const uint64_t *poff, uint32_t k, uint64_t d, uint64_t q,
                       int nthreads, int recompute, uint64_t **offsets_out,
                       uint64_t **positions_out) {
  if (check_params(d, q)) return RKO_EINVAL;
  if (!offsets_out || !positions_out) return RKO_EINVAL;
  if (nthreads < 1) nthreads = 1;
  for (uint32_t j = 0; j < k; ++j)
    if (poff[j + 1] <= poff[j]) return RKO_EINVAL; /* m = 0 is invalid */

  int status = RKO_OK;
  uint64_t *offsets = (uint64_t *)calloc((size_t)k + 1, sizeof(uint64_t));
  uint64_t (*pairs)[2] = NULL;
  lengroup *groups = NULL;
  uint64_t ng = 0;
  worker *ws = NULL;
  pthread_t *th = NULL;
  uint64_t *positions = NULL;
  if (!offsets) return RKO_ENOMEM;

  /* group patterns by length: sort (m, id) pairs */
  if (k > 0) {
    pairs = (uint64_t(*)[2])malloc((size_t)k * sizeof(*pairs));
    groups = (lengroup *)calloc(k, sizeof(lengroup));
    if (!pairs || !groups) { status = RKO_ENOMEM; goto done; }
    for (uint32_t j = 0; j < k; ++j) {
      pairs[j][0] = poff[j + 1] - poff[j];
      pairs[j][1] = j;
    }
    qsort(pairs, k, sizeof(*pairs), cmp_pair);
    for (uint32_t a = 0; a < k;) {
      uint32_t b = a;
      while (b < k && pairs[b][0] == pairs[a][0]) ++b;
      lengroup *g = &groups[ng++];
      g->m = pairs[a][0];
      g->npat = b - a;
      uint64_t (*hp)[2] = (uint64_t(*)[2])malloc((size_t)g->npat * sizeof(*hp));
      g->hash = (uint64_t *)malloc((size_t)g->npat * sizeof(uint64_t));
      g->id = (uint32_t *)malloc((size_t)g->npat * sizeof(uint32_t));
      if (!hp || !g->hash || !g->id) { free(hp); status = RKO_ENOMEM; goto done; }
      for (uint32_t i = a; i < b; ++i) {
        uint32_t id = (uint32_t)pairs[i][1];
        hp[i - a][0] = rko_hash(pbytes + poff[id], g->m, d, q); /* hx */
        hp[i - a][1] = id;
      }
      qsort(hp, g->npat, sizeof(*hp), cmp_pair);
      for (uint64_t i = 0; i < g->npat; ++i) {
        g->hash[i] = hp[i][0];
        g->id[i] = (uint32_t)hp[i][1];
      }
      free(hp);
      a = b;
    }
  }

  {
    ws = (worker *)calloc((size_t)nthreads, sizeof(worker));
    th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!ws || !th) { status = RKO_ENOMEM; goto done; }
    uint64_t span = (n + (uint64_t)nthreads - 1) / (uint64_t)nthreads;
    for (int t = 0; t < nthreads; ++t) {
      worker *w = &ws[t];
      w->text = text; w->n = n; w->pbytes = pbytes; w->poff = poff;
      w->d = d; w->q = q; w->g = groups; w->ng = ng; w->recompute = recompute;
      w->x_begin = span * (uint64_t)t < n ? span * (uint64_t)t : n;
      w->x_end = span * (uint64_t)(t + 1) < n ? span * (uint64_t)(t + 1) : n;
    }
    if (nthreads == 1) {
      run_worker(&ws[0]);
    } else {
      for (int t = 0; t < nthreads; ++t)
        if (pthread_create(&th[t], NULL, run_worker, &ws[t]) != 0) {
          /* fall back: run the remaining parts on this thread */
          for (int u = t; u < nthreads; ++u) { run_worker(&ws[u]); th[u] = 0; }
          for (int u = 0; u < t; ++u) pthread_join(th[u], NULL);
          goto joined;
        }
      for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    joined:;
    }
    for (int t = 0; t < nthreads; ++t)
      if (ws[t].status) { status = ws[t].status; goto done; }

    /* per-pattern counts, then fill in worker order (= ascending x) */
    for (int t = 0; t < nthreads; ++t)
      for (uint64_t i = 0; i < ws[t].out.len; ++i) offsets[ws[t].out.pid[i] + 1]++;
    for (uint32_t j = 0; j < k; ++j) offsets[j + 1] += offsets[j];
    uint64_t total = offsets[k];
    positions = (uint64_t *)malloc((size_t)(total ? total : 1) * sizeof(uint64_t));
    uint64_t *cur = (uint64_t *)malloc(((size_t)k + 1) * sizeof(uint64_t));
    if (!positions || !cur) { free(cur); status = RKO_ENOMEM; goto done; }
    memcpy(cur, offsets, ((size_t)k + 1) * sizeof(uint64_t));
    /* within one worker, hits of one group are in x order but groups are
     * visited one after another; a pattern belongs to a single group, so its
     * hits inside one worker are already ascending. */
    for (int t = 0; t < nthreads; ++t)
      for (uint64_t i = 0; i < ws[t].out.len; ++i) positions[cur[ws[t].out.pid[i]]++] = ws[t].out.pos[i];
    free(cur);
  }

done:
  if (groups) {
    for (uint64_t g = 0; g < ng; ++g) { free(groups[g].hash); free(groups[g].id); }
    free(groups);
  }
  free(pairs);
  if (ws) {
    for (int t = 0; t < nthreads; ++t) hl_free(&ws[t].out);
    free(ws);
  }
  free(th);
  if (status) {
    free(offsets);
    free(positions);
    return status;
  }
  *offsets_out = offsets;
  *positions_out = positions;
  return RKO_OK;
}

int rko_search(const uint8_t *text, uint64_t n, const uint8_t *pbytes, const uint64_t *poff,
               uint32_t k, uint64_t d, uint64_t q, int nthreads, uint64_t **offsets_out,
               uint64_t **positions_out) {
  return search_impl(text, n, pbytes, poff, k, d, q, nthreads, 0, offsets_out, positions_out);
}

int rko_search_recompute(const uint8_t *text, uint64_t n, const uint8_t *pbytes,
                         const uint64_t *poff, uint32_t k, uint64_t d, uint64_t q,
                         uint64_t **offsets_out, uint64_t **positions_out) {
  return search_impl(text, n, pbytes, poff, k, d, q, 1, 1, offsets_out, positions_out);
}

/* The definition: x is an occurrence of P_j iff text[x .. x+m_j) == P_j. */
int rko_brute(const uint8_t *text, uint64_t n, const uint8_t *pbytes, const uint64_t *poff,
              uint32_t k, uint64_t **offsets_out, uint64_t **positions_out) {
  if (!offsets_out || !positions_out) return RKO_EINVAL;
  for (uint32_t j = 0; j < k; ++j)
    if (poff[j + 1] <= poff[j]) return RKO_EINVAL;
  uint64_t *offsets = (uint64_t *)calloc((size_t)k + 1, sizeof(uint64_t));
  if (!offsets) return RKO_ENOMEM;
  hitlist all = {0};
  for (uint32_t j = 0; j < k; ++j) {
    uint64_t m = poff[j + 1] - poff[j];
    uint64_t c = 0;
    if (m <= n)
      for (uint64_t x = 0; x + m <= n; ++x) {
        uint64_t i = 0;
        while (i < m && text[x + i] == pbytes[poff[j] + i]) ++i;
        if (i == m) {
          if (hl_push(&all, j, x)) { hl_free(&all); free(offsets); return RKO_ENOMEM; }
          ++c;
        }
      }
    offsets[j + 1] = offsets[j] + c;
  }
  uint64_t *positions = (uint64_t *)malloc((size_t)(all.len ? all.len : 1) * sizeof(uint64_t));
  if (!positions) { hl_free(&all); free(offsets); return RKO_ENOMEM; }
  if (all.len) memcpy(positions, all.pos, (size_t)all.len * sizeof(uint64_t));
  hl_free(&all);
  *offsets_out = offsets;
  *positions_out = positions;
  return RKO_OK;
}

void rko_free(void *p) { free(p); }
