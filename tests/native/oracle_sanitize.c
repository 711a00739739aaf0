/* Oracle under AddressSanitizer / UndefinedBehaviorSanitizer: random texts
 * and pattern sets over small and large alphabets, the rolling search (1 and
 * 4 threads) and the recompute search checked against brute force, and window
 * hashes checked against a direct big-endian evaluation.  Exit status 0 when
 * every case agrees. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int rko_search(const uint8_t *text, uint64_t n, const uint8_t *pbytes, const uint64_t *poff, uint32_t k,
               uint64_t d, uint64_t q, int nthreads, uint64_t **offsets_out, uint64_t **positions_out);
int rko_search_recompute(const uint8_t *text, uint64_t n, const uint8_t *pbytes, const uint64_t *poff,
                         uint32_t k, uint64_t d, uint64_t q, uint64_t **offsets_out, uint64_t **positions_out);
int rko_brute(const uint8_t *text, uint64_t n, const uint8_t *pbytes, const uint64_t *poff, uint32_t k,
              uint64_t **offsets_out, uint64_t **positions_out);
int rko_window_hashes(const uint8_t *text, uint64_t n, uint64_t m, uint64_t d, uint64_t q, const uint64_t *xs,
                      uint64_t cnt, uint64_t *out);
void rko_free(void *p);

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t rnd(void) { /* xorshift64* */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return rng_state * 2685821657736338717ull;
}

static int same(const uint64_t *ao, const uint64_t *ap, const uint64_t *bo, const uint64_t *bp, uint32_t k) {
  if (memcmp(ao, bo, (k + 1) * sizeof(uint64_t)) != 0) return 0;
  return memcmp(ap, bp, ao[k] * sizeof(uint64_t)) == 0;
}

int main(void) {
  const uint64_t Q = (1ull << 61) - 1;
  static const int alpha[4] = {2, 4, 26, 256};
  for (int trial = 0; trial < 200; ++trial) {
    const int a = alpha[trial % 4];
    const uint64_t n = rnd() % 3000;
    uint8_t *text = (uint8_t *)malloc(n ? n : 1);
    for (uint64_t i = 0; i < n; ++i) text[i] = (uint8_t)(a == 256 ? rnd() & 255 : 'a' + rnd() % a);
    const uint32_t k = (uint32_t)(rnd() % 9);
    uint64_t poff[10];
    uint8_t pbytes[9 * 64];
    poff[0] = 0;
    for (uint32_t j = 0; j < k; ++j) {
      const uint64_t m = 1 + rnd() % 20;
      for (uint64_t i = 0; i < m; ++i) {
        if (n >= m && (rnd() & 1)) {
          pbytes[poff[j] + i] = text[(trial * 7 + j * 13) % (n - m + 1) + i];
        } else {
          pbytes[poff[j] + i] = (uint8_t)(a == 256 ? rnd() & 255 : 'a' + rnd() % a);
        }
      }
      poff[j + 1] = poff[j] + m;
    }
    uint64_t *bo, *bp, *ro, *rp, *to, *tp, *co, *cp;
    if (rko_brute(text, n, pbytes, poff, k, &bo, &bp)) return 2;
    if (rko_search(text, n, pbytes, poff, k, 256, Q, 1, &ro, &rp)) return 3;
    if (rko_search(text, n, pbytes, poff, k, 256, Q, 4, &to, &tp)) return 4;
    if (rko_search_recompute(text, n, pbytes, poff, k, 256, Q, &co, &cp)) return 5;
    if (!same(bo, bp, ro, rp, k) || !same(bo, bp, to, tp, k) || !same(bo, bp, co, cp, k)) {
      fprintf(stderr, "trial %d: search differs from brute force\n", trial);
      return 1;
    }
    rko_free(bo); rko_free(bp); rko_free(ro); rko_free(rp);
    rko_free(to); rko_free(tp); rko_free(co); rko_free(cp);
    /* window hashes of m <= 7 bytes are the big-endian integer itself */
    if (n >= 7) {
      uint64_t xs[8], out[8];
      const uint64_t m = 1 + rnd() % 7;
      for (int i = 0; i < 8; ++i) xs[i] = rnd() % (n - m + 1);
      if (rko_window_hashes(text, n, m, 256, Q, xs, 8, out)) return 6;
      for (int i = 0; i < 8; ++i) {
        uint64_t be = 0;
        for (uint64_t j = 0; j < m; ++j) be = (be << 8) | text[xs[i] + j];
        if (be != out[i]) {
          fprintf(stderr, "trial %d: window hash differs\n", trial);
          return 1;
        }
      }
    }
    free(text);
  }
  printf("ok\n");
  return 0;
}
