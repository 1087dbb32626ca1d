// Host number theory for the library: modular powers with 128-bit products,
// deterministic Miller-Rabin, primitive roots, roots of unity and Shoup
// constants W' = floor(W beta / p) (Algorithm 2 input conditions).
#pragma once

#include <stdint.h>

#include <vector>

namespace hntt {

using u128 = unsigned __int128;

// a b mod m (a 64-bit division when all three are below 2^32)
inline uint64_t mulmod(uint64_t a, uint64_t b, uint64_t m) {
  if ((a | b | m) >> 32 == 0) return a * b % m;
  return (uint64_t)((u128)a * b % m);
}

inline uint64_t powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  for (; e; e >>= 1) {
    if (e & 1) r = mulmod(r, a, m);
    a = mulmod(a, a, m);
  }
  return r;
}

// Deterministic for all 64-bit n with the first twelve prime bases.
inline bool is_prime_u64(uint64_t n) {
  static const uint64_t kBases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return false;
  for (uint64_t b : kBases) {
    if (n % b == 0) return n == b;
  }
  uint64_t d = n - 1;
  int s = 0;
  while (!(d & 1)) {
    d >>= 1;
    ++s;
  }
  for (uint64_t a : kBases) {
    uint64_t x = powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool witness = true;
    for (int r = 1; r < s && witness; ++r) {
      x = mulmod(x, x, n);
      if (x == n - 1) witness = false;
    }
    if (witness) return false;
  }
  return true;
}

// Distinct prime factors by trial division up to the square root of the
// remaining cofactor, with Miller-Rabin to stop early on a prime cofactor.
inline std::vector<uint64_t> prime_factors(uint64_t n) {
  std::vector<uint64_t> f;
  bool cofactor_prime = is_prime_u64(n);
  for (uint64_t q = 2; !cofactor_prime && q * q <= n; q += (q == 2 ? 1 : 2)) {
    if (n % q == 0) {
      f.push_back(q);
      while (n % q == 0) n /= q;
      cofactor_prime = is_prime_u64(n);
    }
  }
  if (n > 1) f.push_back(n);
  return f;
}

// Smallest g with g^((p-1)/q) != 1 for every prime q | p - 1; 0 if p is not an odd prime.
inline uint64_t primitive_root(uint64_t p) {
  if (p < 3 || !is_prime_u64(p)) return 0;
  const std::vector<uint64_t> f = prime_factors(p - 1);
  for (uint64_t g = 2; g < p; ++g) {
    bool ok = true;
    for (uint64_t q : f)
      if (powmod(g, (p - 1) / q, p) == 1) {
        ok = false;
        break;
      }
    if (ok) return g;
  }
  return 0;
}

// floor(w * 2^bits / p) for w < p < 2^bits, bits in {32, 64}.
inline uint64_t shoup_constant(uint64_t w, uint64_t p, int bits) {
  if (bits == 32) return (w << 32) / p;
  return (uint64_t)(((u128)w << bits) / p);
}

// Largest prime below 2^bits that is 1 mod 2^v (0 if none).
inline uint64_t find_prime(unsigned bits, unsigned v) {
  if (bits < 2 || bits > 64 || v >= bits) return 0;
  const uint64_t top = bits == 64 ? ~0ull : ((1ull << bits) - 1);
  const uint64_t step = 1ull << v;
  for (uint64_t k = (top - 1) / step; k > 0; --k) {
    const uint64_t c = k * step + 1;
    if (is_prime_u64(c)) return c;
  }
  return 0;
}

inline unsigned bitrev(unsigned x, int bits) {
  unsigned r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

}  // namespace hntt
