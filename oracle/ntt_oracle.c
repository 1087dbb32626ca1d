/*
 * Plain, slow CPU oracle for the number-theoretic transform of
 * Harvey, "Faster arithmetic for number-theoretic transforms" (arXiv:1205.2926).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product: only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no source with the GPU library and must never be
 * linked into it.
 *
 * Every operation in F_p is fully reduced to [0, p) immediately (no lazy or
 * redundant representations, no Shoup or Montgomery constants): additions use
 * one compare-and-subtract, multiplications use the hardware remainder of the
 * exact double-width product.  Words are held as uint64_t for both the 30-bit
 * and the 62-bit primes.
 *
 * Passages followed (section / algorithm / equation of the paper):
 *   - the NTT definition b_j = sum_i omega^{ij} a_i          (Section 1, display eq.)
 *   - the in-place radix-2 FFT with bit-reversed output       (Section 1, Algorithm 1)
 *   - the inverse as Algorithm 1 run backwards, giving the
 *     butterfly (X, Y) -> (X + W Y, X - W Y)                  (Section 4, first paragraph)
 *   - the problem setting: p prime, L = 2^l divides p - 1     (Section 1)
 *   - large-integer multiplication, the application that
 *     motivates fast transforms                               (Section 1, first paragraph)
 *
 * Parity pins for every function live in tests/oracle_pins.py; no
 * function here is "parity unpinned".
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ---------------- F_p arithmetic, fully reduced after every operation ---------------- */

static uint64_t add_mod(uint64_t a, uint64_t b, uint64_t p) {
  uint64_t s = a + b; /* a, b < p < 2^63: no overflow */
  if (s >= p) s -= p;
  return s;
}

static uint64_t sub_mod(uint64_t a, uint64_t b, uint64_t p) {
  return (a >= b) ? a - b : a + (p - b);
}

static uint64_t mul_mod(uint64_t a, uint64_t b, uint64_t p) {
  if (p <= 0xFFFFFFFFull) return (a * b) % p; /* a, b < 2^32: product fits 64 bits */
  return (uint64_t)(((u128)a * b) % p);
}

uint64_t oracle_pow_mod(uint64_t a, uint64_t e, uint64_t p) {
  uint64_t r = 1 % p;
  a %= p;
  while (e) {
    if (e & 1) r = mul_mod(r, a, p);
    a = mul_mod(a, a, p);
    e >>= 1;
  }
  return r;
}

/* Inverse by Fermat's little theorem (p prime). */
uint64_t oracle_inv_mod(uint64_t a, uint64_t p) { return oracle_pow_mod(a, p - 2, p); }

/* ---------------- number theory for the problem setting (Section 1) ---------------- */

/* Deterministic Miller-Rabin for 64-bit n: the first twelve primes as bases
 * are a proven witness set for every n < 3.3e24. */
int oracle_is_prime(uint64_t n) {
  static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; ++i) {
    if (n == bases[i]) return 1;
    if (n % bases[i] == 0) return 0;
  }
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (int i = 0; i < 12; ++i) {
    uint64_t x = oracle_pow_mod(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int composite = 1;
    for (int r = 1; r < s; ++r) {
      x = mul_mod(x, x, n);
      if (x == n - 1) { composite = 0; break; }
    }
    if (composite) return 0;
  }
  return 1;
}

/* Distinct prime factors of n by trial division.  Returns their count. */
static int distinct_prime_factors(uint64_t n, uint64_t *out, int cap) {
  int k = 0;
  for (uint64_t f = 2; f * f <= n; f += (f == 2 ? 1 : 2)) {
    if (n % f == 0) {
      if (k < cap) out[k] = f;
      ++k;
      while (n % f == 0) n /= f;
    }
  }
  if (n > 1) {
    if (k < cap) out[k] = n;
    ++k;
  }
  return k;
}

/* Smallest primitive root of the prime p: g generates F_p^* iff
 * g^((p-1)/q) != 1 for every prime q dividing p - 1.  Returns 0 on failure. */
uint64_t oracle_primitive_root(uint64_t p) {
  uint64_t f[64];
  int k = distinct_prime_factors(p - 1, f, 64);
  if (k > 64) return 0;
  for (uint64_t g = 2; g < p; ++g) {
    int ok = 1;
    for (int i = 0; i < k && ok; ++i)
      if (oracle_pow_mod(g, (p - 1) / f[i], p) == 1) ok = 0;
    if (ok) return g;
  }
  return 0;
}

/* omega = g^((p-1)/L): a primitive L-th root of unity when g is a primitive
 * root and L | p - 1.  Returns 0 when L does not divide p - 1. */
uint64_t oracle_root_of_unity(uint64_t p, uint64_t g, unsigned log2_len) {
  uint64_t L = 1ull << log2_len;
  if ((p - 1) % L) return 0;
  return oracle_pow_mod(g, (p - 1) / L, p);
}

/* Largest prime p < 2^bits with p = 1 (mod 2^v), by downward search over the
 * candidates k * 2^v + 1 with the deterministic Miller-Rabin test above. */
uint64_t oracle_largest_ntt_prime(unsigned bits, unsigned v) {
  uint64_t step = 1ull << v;
  uint64_t k = ((bits >= 64 ? ~0ull : ((1ull << bits) - 1)) - 1) / step;
  for (; k > 0; --k) {
    uint64_t c = k * step + 1;
    if (oracle_is_prime(c)) return c;
  }
  return 0;
}

/* ---------------- the transform (Section 1, Algorithm 1) ---------------- */

/* Forward NTT in place: natural-order input in [0,p), output b_j stored at
 * position rev_l(j), fully reduced.  Stage i = 1..l uses zeta = omega^(2^(i-1))
 * and half-distance m = 2^(l-i); the butterfly on (x[t+k], x[t+k+m]) with
 * t = 2jm is (X, Y) -> (X + Y, zeta^k (X - Y)). */
void oracle_ntt_forward(uint64_t *x, unsigned l, uint64_t p, uint64_t omega) {
  for (unsigned i = 1; i <= l; ++i) {
    uint64_t zeta = oracle_pow_mod(omega, 1ull << (i - 1), p);
    size_t m = (size_t)1 << (l - i);
    size_t nblocks = (size_t)1 << (i - 1);
    for (size_t j = 0; j < nblocks; ++j) {
      size_t t = 2 * j * m;
      uint64_t w = 1; /* zeta^k, k = 0 */
      for (size_t k = 0; k < m; ++k) {
        uint64_t X = x[t + k], Y = x[t + k + m];
        x[t + k] = add_mod(X, Y, p);
        x[t + k + m] = mul_mod(w, sub_mod(X, Y, p), p);
        w = mul_mod(w, zeta, p);
      }
    }
  }
}

/* Inverse NTT in place: Algorithm 1 run backwards (stages i = l..1) with the
 * butterfly (X, Y) -> (X + W Y, X - W Y), W = zeta^(-k), which undoes stage i
 * up to a factor 2; the accumulated factor L is removed by multiplying every
 * entry by L^(-1).  Bit-reversed input, natural-order output in [0,p). */
void oracle_ntt_inverse(uint64_t *x, unsigned l, uint64_t p, uint64_t omega) {
  uint64_t omega_inv = oracle_inv_mod(omega, p);
  for (unsigned i = l; i >= 1; --i) {
    uint64_t zeta = oracle_pow_mod(omega_inv, 1ull << (i - 1), p);
    size_t m = (size_t)1 << (l - i);
    size_t nblocks = (size_t)1 << (i - 1);
    for (size_t j = 0; j < nblocks; ++j) {
      size_t t = 2 * j * m;
      uint64_t w = 1;
      for (size_t k = 0; k < m; ++k) {
        uint64_t X = x[t + k];
        uint64_t S = mul_mod(w, x[t + k + m], p);
        x[t + k] = add_mod(X, S, p);
        x[t + k + m] = sub_mod(X, S, p);
        w = mul_mod(w, zeta, p);
      }
    }
  }
  size_t L = (size_t)1 << l;
  uint64_t Linv = oracle_inv_mod((uint64_t)(L % p), p);
  for (size_t n = 0; n < L; ++n) x[n] = mul_mod(x[n], Linv, p);
}

/* Batch forms: count transforms of length 2^l laid out back to back. */
void oracle_ntt_forward_batch(uint64_t *x, size_t count, unsigned l, uint64_t p, uint64_t omega) {
  for (size_t b = 0; b < count; ++b) oracle_ntt_forward(x + (b << l), l, p, omega);
}
void oracle_ntt_inverse_batch(uint64_t *x, size_t count, unsigned l, uint64_t p, uint64_t omega) {
  for (size_t b = 0; b < count; ++b) oracle_ntt_inverse(x + (b << l), l, p, omega);
}

/* One output of the definition (Section 1, display eq.), straight from the
 * sum: b_j = sum_{i<L} omega^(i j) a_i mod p.  O(L) per call, for checking
 * sampled outputs of long transforms. */
uint64_t oracle_dft_point(const uint64_t *a, unsigned l, uint64_t p, uint64_t omega, uint64_t j) {
  size_t L = (size_t)1 << l;
  uint64_t wj = oracle_pow_mod(omega, j, p);
  uint64_t w = 1, acc = 0;
  for (size_t i = 0; i < L; ++i) {
    acc = add_mod(acc, mul_mod(w, a[i] % p, p), p);
    w = mul_mod(w, wj, p);
  }
  return acc;
}

/* Bit reversal of the low l bits. */
uint64_t oracle_bitrev(uint64_t j, unsigned l) {
  uint64_t r = 0;
  for (unsigned b = 0; b < l; ++b) r |= ((j >> b) & 1ull) << (l - 1 - b);
  return r;
}

/* ---------------- applications: polynomial products (Section 1, motivation) ---------------- */

/* c_i = a_i b_i mod p. */
void oracle_pointwise(const uint64_t *a, const uint64_t *b, uint64_t *c, size_t n, uint64_t p) {
  for (size_t i = 0; i < n; ++i) c[i] = mul_mod(a[i] % p, b[i] % p, p);
}

/* Product of two polynomials mod p by the convolution theorem: zero-pad both
 * to L = 2^l >= na + nb - 1, forward NTT (bit-reversed), pointwise product,
 * inverse NTT (bit-reversed in, natural out), keep na + nb - 1 coefficients.
 * omega must be a primitive 2^l-th root of unity.  Returns -1 if L is short. */
int oracle_polymul_mod(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *c,
                       unsigned l, uint64_t p, uint64_t omega) {
  size_t L = (size_t)1 << l;
  if (na == 0 || nb == 0 || na + nb - 1 > L) return -1;
  uint64_t *fa = (uint64_t *)calloc(L, sizeof(uint64_t));
  uint64_t *fb = (uint64_t *)calloc(L, sizeof(uint64_t));
  if (!fa || !fb) { free(fa); free(fb); return -2; }
  for (size_t i = 0; i < na; ++i) fa[i] = a[i] % p;
  for (size_t i = 0; i < nb; ++i) fb[i] = b[i] % p;
  oracle_ntt_forward(fa, l, p, omega);
  oracle_ntt_forward(fb, l, p, omega);
  oracle_pointwise(fa, fb, fa, L, p);
  oracle_ntt_inverse(fa, l, p, omega);
  memcpy(c, fa, (na + nb - 1) * sizeof(uint64_t));
  free(fa);
  free(fb);
  return 0;
}

/* Chinese remaindering for three pairwise coprime moduli below 2^31, by the
 * textbook formula x = sum_k r_k M_k (M_k^(-1) mod q_k) mod M, M = q1 q2 q3,
 * in 128-bit integers (every term is below 2^122).  The result is returned
 * mod 2^64; it is the exact integer whenever that is below 2^64. */
void oracle_crt3(const uint64_t *r1, const uint64_t *r2, const uint64_t *r3, uint64_t *out, size_t n,
                 uint64_t q1, uint64_t q2, uint64_t q3) {
  u128 M = (u128)q1 * q2 * q3;
  u128 M1 = (u128)q2 * q3, M2 = (u128)q1 * q3, M3 = (u128)q1 * q2;
  u128 y1 = oracle_inv_mod((uint64_t)(M1 % q1), q1);
  u128 y2 = oracle_inv_mod((uint64_t)(M2 % q2), q2);
  u128 y3 = oracle_inv_mod((uint64_t)(M3 % q3), q3);
  for (size_t i = 0; i < n; ++i) {
    u128 x = ((u128)r1[i] * y1 % q1) * M1 + ((u128)r2[i] * y2 % q2) * M2 + ((u128)r3[i] * y3 % q3) * M3;
    out[i] = (uint64_t)(x % M);
  }
}

/* Exact integer product by the schoolbook sum c_k = sum_i a_i b_(k-i),
 * accumulated mod 2^64 (exact when every c_k < 2^64). */
void oracle_schoolbook(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, uint64_t *c) {
  if (na == 0 || nb == 0) return;
  memset(c, 0, (na + nb - 1) * sizeof(uint64_t));
  for (size_t i = 0; i < na; ++i)
    for (size_t j = 0; j < nb; ++j) c[i + j] += a[i] * b[j];
}

/* One exact product coefficient c_k = sum_i a_i b_(k-i), O(min(na, nb)). */
uint64_t oracle_product_coeff(const uint64_t *a, size_t na, const uint64_t *b, size_t nb, size_t k) {
  uint64_t acc = 0;
  size_t lo = (k + 1 > nb) ? k + 1 - nb : 0;
  size_t hi = (k < na - 1) ? k : na - 1;
  for (size_t i = lo; i <= hi; ++i) acc += a[i] * b[k - i];
  return acc;
}

/* p(r) mod m for the polynomial with coefficients c[0..n) (Horner's rule), for
 * checking long products by evaluation at a random point (Schwartz-Zippel):
 * (a b)(r) = a(r) b(r) mod m. */
uint64_t oracle_poly_eval(const uint64_t *c, size_t n, uint64_t r, uint64_t m) {
  uint64_t acc = 0;
  for (size_t i = n; i-- > 0;) acc = add_mod(mul_mod(acc, r % m, m), c[i] % m, m);
  return acc;
}

/* Long multiplication of non-negative integers given as little-endian base-2^32
 * limbs (the schoolbook method, with one carry pass per row): out[0..na+nb) =
 * a * b.  Every partial sum out[i+j] + a_i b_j + carry is below 2^64, since
 * (2^32 - 1)^2 + 2 (2^32 - 1) = 2^64 - 1.  Used to pin large-integer products. */
void oracle_bigmul_schoolbook(const uint32_t *a, size_t na, const uint32_t *b, size_t nb, uint32_t *out) {
  memset(out, 0, (na + nb) * sizeof(uint32_t));
  for (size_t i = 0; i < na; ++i) {
    uint64_t carry = 0;
    for (size_t j = 0; j < nb; ++j) {
      const uint64_t t = (uint64_t)a[i] * b[j] + out[i + j] + carry;
      out[i + j] = (uint32_t)t;
      carry = t >> 32;
    }
    out[i + nb] = (uint32_t)carry;
  }
}

/* The integer given by n little-endian base-2^32 limbs, reduced mod m (Horner's
 * rule from the most significant limb; m < 2^63). */
uint64_t oracle_limbs_mod(const uint32_t *x, size_t n, uint64_t m) {
  const uint64_t base = (uint64_t)(((u128)1 << 32) % m);
  uint64_t acc = 0;
  for (size_t i = n; i-- > 0;) acc = add_mod(mul_mod(acc, base, m), (uint64_t)x[i] % m, m);
  return acc;
}
