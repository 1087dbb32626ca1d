/*
 * Same-host counterpart of Table 1 (Section 5): one forward transform of
 * length 2^11 over a 62-bit prime on one CPU core, with the butterfly of
 * Algorithm 2 (fully reducing) and of Algorithm 3 (lazy), W and W' read from a
 * precomputed table, in the stage order of Algorithm 1 (natural order in,
 * bit-reversed out).  Table 1 reports total transform time divided by the
 * number of butterflies (l * 2^(l-1), W = 1 butterflies included); t1_time
 * returns the same quantity in nanoseconds and in time-stamp-counter ticks.
 *
 * This is a measurement program for the host CPU, separate from the GPU
 * library; its transforms are checked against the oracle by the CPU tests.
 */
#define _POSIX_C_SOURCE 199309L
#include <stdint.h>
#include <stdlib.h>
#include <time.h>
#include <x86intrin.h>

typedef unsigned __int128 u128;

static uint64_t mulmod(uint64_t a, uint64_t b, uint64_t p) { return (uint64_t)((u128)a * b % p); }

/* Per-stage table: for the stage whose butterflies pair elements m apart,
 * entries [m, 2m) hold (W, W') for W = omega^(k L / (2m)), k < m, so the
 * twiddles of one stage are contiguous.  W' = floor(W 2^64 / p). */
typedef struct {
  uint64_t p;
  int l;
  uint64_t *w, *wp;
} t1_plan;

t1_plan *t1_plan_create(uint64_t p, uint64_t omega, int l) {
  t1_plan *pl = (t1_plan *)malloc(sizeof(t1_plan));
  const size_t L = (size_t)1 << l;
  pl->p = p;
  pl->l = l;
  pl->w = (uint64_t *)malloc(L * sizeof(uint64_t));
  pl->wp = (uint64_t *)malloc(L * sizeof(uint64_t));
  for (size_t m = 1; m < L; m <<= 1) {
    uint64_t root = omega;  /* omega^(L / (2m)) */
    for (size_t e = L / (2 * m); e > 1; e >>= 1) root = mulmod(root, root, p);
    uint64_t w = 1;
    for (size_t k = 0; k < m; ++k) {
      pl->w[m + k] = w;
      pl->wp[m + k] = (uint64_t)(((u128)w << 64) / p);
      w = mulmod(w, root, p);
    }
  }
  return pl;
}

void t1_plan_destroy(t1_plan *pl) {
  free(pl->w);
  free(pl->wp);
  free(pl);
}

/* Word arithmetic shared by both butterflies.  x >= m ? x - m : x without a
 * branch (x - m wraps above x exactly when x < m). */
static inline uint64_t csub64(uint64_t x, uint64_t m) {
  const uint64_t d = x - m;
  return d < x ? d : x;
}

/* Shoup's product: for any t < 2^64 and W' = floor(W 2^64 / p), the quotient
 * estimate Q = hi(W' t) leaves W t - Q p in [0, 2p); only the low words of the two
 * products are needed. */
static inline uint64_t shoup64(uint64_t t, uint64_t w, uint64_t wp, uint64_t p) {
  const uint64_t q = (uint64_t)(((u128)wp * t) >> 64);
  return w * t - q * p;
}

/* Algorithm 2 (fully reducing): X, Y in [0,p) -> X + Y mod p and W (X - Y) mod p.
 * The difference is taken mod p as the smaller of X - Y and X - Y + p (wrapping
 * arithmetic), the product is reduced once more from [0,2p). */
static inline void bfly2(uint64_t *x, uint64_t *y, uint64_t w, uint64_t wp, uint64_t p) {
  const uint64_t d = *x - *y, dp = d + p;
  const uint64_t diff = dp < d ? dp : d;
  *x = csub64(*x + *y, p);
  *y = csub64(shoup64(diff, w, wp, p), p);
}

/* Algorithm 3 (lazy): X, Y in [0,2p) -> X + Y and W (X - Y), both kept in [0,2p)
 * (p < 2^62): one conditional subtraction of 2p from the sum, none after the
 * product, whose input X - Y + 2p lies in (0, 4p). */
static inline void bfly3(uint64_t *x, uint64_t *y, uint64_t w, uint64_t wp, uint64_t p2) {
  const uint64_t t = *x - *y + p2;
  *x = csub64(*x + *y, p2);
  *y = shoup64(t, w, wp, p2 >> 1);
}

/* One forward transform in place with Algorithm `alg` (2 or 3); lazy results
 * are left in [0,2p) (the caller reduces them if it needs [0,p)). */
void t1_forward(const t1_plan *pl, int alg, uint64_t *x) {
  const uint64_t p = pl->p, p2 = 2 * p;
  const size_t L = (size_t)1 << pl->l;
  for (size_t m = L / 2; m >= 1; m >>= 1) {
    const uint64_t *w = pl->w + m, *wp = pl->wp + m;
    for (size_t t = 0; t < L; t += 2 * m) {
      uint64_t *u = x + t, *v = x + t + m;
      if (alg == 2) {
        for (size_t k = 0; k < m; ++k) bfly2(u + k, v + k, w[k], wp[k], p);
      } else {
        for (size_t k = 0; k < m; ++k) bfly3(u + k, v + k, w[k], wp[k], p2);
      }
    }
  }
}

/* Time `reps` transforms of x with Algorithm `alg`; per butterfly: *ns and *ticks (TSC). */
void t1_time(const t1_plan *pl, int alg, uint64_t *x, int reps, double *ns, double *ticks) {
  struct timespec a, b;
  t1_forward(pl, alg, x);  /* warm the caches */
  clock_gettime(CLOCK_MONOTONIC, &a);
  const uint64_t c0 = __rdtsc();
  for (int r = 0; r < reps; ++r) t1_forward(pl, alg, x);
  const uint64_t c1 = __rdtsc();
  clock_gettime(CLOCK_MONOTONIC, &b);
  const double bfly = (double)reps * pl->l * (double)((size_t)1 << (pl->l - 1));
  *ns = ((b.tv_sec - a.tv_sec) * 1e9 + (b.tv_nsec - a.tv_nsec)) / bfly;
  *ticks = (double)(c1 - c0) / bfly;
}
