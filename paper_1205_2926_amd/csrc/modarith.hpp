// Device word arithmetic and the butterflies of arXiv:1205.2926 for gfx950.
//
// Words are 32-bit (beta = 2^32: one v_mul_hi_u32 / v_mul_lo_u32 each) or
// 64-bit (beta = 2^64: the high and low halves of 64x64-bit products are
// assembled from 32x32->64-bit partial products).  No MFMA: the butterfly is
// not a dense contraction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hntt {

struct Word32 {
  using T = uint32_t;
  static constexpr int kBits = 32;
  __device__ __forceinline__ static T mulhi(T a, T b) { return __umulhi(a, b); }
  __device__ __forceinline__ static T mullo(T a, T b) { return a * b; }
};

struct Word64 {
  using T = uint64_t;
  static constexpr int kBits = 64;
  // floor(a*b / 2^64) from the four 32x32->64 partial products; every partial
  // sum below stays under 2^64, and the last one is exactly the high word.
  __device__ __forceinline__ static T mulhi(T a, T b) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t p00 = (uint64_t)a0 * b0;
    const uint64_t p01 = (uint64_t)a0 * b1 + (p00 >> 32);
    const uint64_t p10 = (uint64_t)a1 * b0 + (uint32_t)p01;
    return (uint64_t)a1 * b1 + (p01 >> 32) + (p10 >> 32);
  }
  // a*b mod 2^64: one full 32x32 product plus the low halves of the cross terms.
  __device__ __forceinline__ static T mullo(T a, T b) {
    const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
    const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
    const uint64_t p00 = (uint64_t)a0 * b0;
    const uint32_t cross = a0 * b1 + a1 * b0;
    return p00 + ((uint64_t)cross << 32);
  }
};

// x >= m ? x - m : x, branch-free (unsigned wrap makes x - m > x when x < m).
template <class T>
__device__ __forceinline__ T csub(T x, T m) {
  const T d = x - m;
  return d < x ? d : x;
}

// -p mod 2^32 for the multiply-add below, behind an empty asm statement so that the
// compiler cannot see it is a negation (it would otherwise rewrite Q (beta - p) + W t
// as W t - Q p: two low products and a subtraction).  The statement has no side
// effects, so the compiler computes it once per kernel (one vector register).
__device__ __forceinline__ uint32_t opaque_neg_u32(uint32_t p) {
  uint32_t np = 0u - p;
  asm("; -p %0" : "+v"(np));
  return np;
}

// Shoup's product by a constant (Algorithm 2, estimated quotient then two
// low products): for any 0 <= t < beta and W' = floor(W beta / p),
// W t - Q p lies in [0, 2p) (Theorem 1), so no correction is applied here.
// On 32-bit words the low words come from one v_mul_lo_u32 (W t) and one
// v_mad_u64_u32: Q (beta - p) + W t, whose low word is W t - Q p mod beta.
template <class Wd>
__device__ __forceinline__ typename Wd::T shoup_lazy(typename Wd::T t, typename Wd::T w, typename Wd::T wp,
                                                     typename Wd::T p) {
  if constexpr (Wd::kBits == 32) {
    const uint32_t q = Wd::mulhi(wp, t);
    const uint32_t wt = w * t;
    return (uint32_t)((uint64_t)q * opaque_neg_u32(p) + wt);
  } else {
    const typename Wd::T q = Wd::mulhi(wp, t);
    return Wd::mullo(w, t) - Wd::mullo(q, p);
  }
}

// The same product with the low words from two v_mul_lo_u32 and a subtraction
// (Algorithm 2's steps as written).  The inverse passes use this form: with the
// multiply-add form their row and column passes measured slower.
template <class Wd>
__device__ __forceinline__ typename Wd::T shoup_lazy_sub(typename Wd::T t, typename Wd::T w, typename Wd::T wp,
                                                         typename Wd::T p) {
  const typename Wd::T q = Wd::mulhi(wp, t);
  return Wd::mullo(w, t) - Wd::mullo(q, p);
}

// Montgomery's product (the multiplication of Algorithm 5): for 0 <= t < beta,
// W' = W beta mod p in [0,p) and J = p^-1 mod beta, the high word R1 of W' t is
// below p; Q = (W' t mod beta) J mod beta makes Q p agree with W' t in the low
// word, so W' t - Q p = beta (R1 - H) with H = floor(Q p / beta) < p, and
// R1 - H + p lies in (0, 2p) and is congruent to W t mod p.
template <class Wd>
__device__ __forceinline__ typename Wd::T mont_lazy(typename Wd::T t, typename Wd::T wm, typename Wd::T p,
                                                    typename Wd::T j) {
  using T = typename Wd::T;
  const T r0 = Wd::mullo(wm, t);
  const T r1 = Wd::mulhi(wm, t);
  const T q = Wd::mullo(r0, j);
  return r1 - Wd::mulhi(q, p) + p;
}

// Algorithm 3 (lazy forward butterfly): X, Y in [0,2p), p < beta/4.
// X' = X + Y reduced once to [0,2p); T = X - Y + 2p in [0,4p); Y' = W T in [0,2p).
template <class Wd>
__device__ __forceinline__ void bfly_fwd_lazy(typename Wd::T &x, typename Wd::T &y, typename Wd::T w,
                                              typename Wd::T wp, typename Wd::T p, typename Wd::T p2) {
  using T = typename Wd::T;
  const T s = csub<T>(x + y, p2);
  const T t = x - y + p2;
  y = shoup_lazy<Wd>(t, w, wp, p);
  x = s;
}

// Algorithm 5 (Montgomery forward butterfly): X, Y in [0,2p), p < beta/4, the
// twiddle given only as W' = W beta mod p.  X' as in Algorithm 3; Y' = W T in [0,2p).
template <class Wd>
__device__ __forceinline__ void bfly_fwd_mont(typename Wd::T &x, typename Wd::T &y, typename Wd::T wm,
                                              typename Wd::T p, typename Wd::T p2, typename Wd::T j) {
  using T = typename Wd::T;
  const T s = csub<T>(x + y, p2);
  const T t = x - y + p2;
  y = mont_lazy<Wd>(t, wm, p, j);
  x = s;
}

// Forward butterfly with W = 1 in the lazy range: X' as above, Y' = X - Y + 2p
// reduced once to [0,2p).
template <class Wd>
__device__ __forceinline__ void bfly_fwd_lazy_w1(typename Wd::T &x, typename Wd::T &y, typename Wd::T p2) {
  using T = typename Wd::T;
  const T s = csub<T>(x + y, p2);
  const T t = csub<T>(x - y + p2, p2);
  x = s;
  y = t;
}

// Algorithm 2 (plain forward butterfly): X, Y in [0,p), p < beta/2, every
// output fully reduced.  The signed test T < 0 is done unsigned: with
// d = X - Y mod beta, min(d, d + p) is X - Y mod p.
template <class Wd>
__device__ __forceinline__ void bfly_fwd_plain(typename Wd::T &x, typename Wd::T &y, typename Wd::T w,
                                               typename Wd::T wp, typename Wd::T p) {
  using T = typename Wd::T;
  const T s = csub<T>(x + y, p);
  T d = x - y;
  const T dp = d + p;
  d = dp < d ? dp : d;
  y = csub<T>(shoup_lazy<Wd>(d, w, wp, p), p);
  x = s;
}

template <class Wd>
__device__ __forceinline__ void bfly_fwd_plain_w1(typename Wd::T &x, typename Wd::T &y, typename Wd::T p) {
  using T = typename Wd::T;
  const T s = csub<T>(x + y, p);
  T d = x - y;
  const T dp = d + p;
  y = dp < d ? dp : d;
  x = s;
}

// Algorithm 4 (lazy inverse butterfly): X, Y in [0,4p), p < beta/4.
// X reduced once to [0,2p); T = W Y in [0,2p); X' = X + T, Y' = X - T + 2p in [0,4p).
template <class Wd>
__device__ __forceinline__ void bfly_inv_lazy(typename Wd::T &x, typename Wd::T &y, typename Wd::T w,
                                              typename Wd::T wp, typename Wd::T p, typename Wd::T p2) {
  using T = typename Wd::T;
  const T xr = csub<T>(x, p2);
  const T t = shoup_lazy_sub<Wd>(y, w, wp, p);
  x = xr + t;
  y = xr - t + p2;
}

// Inverse butterfly of the lazy [0,4p) range with Montgomery's product in place
// of Shoup's (Section 4 notes that the lazy idea carries over to other modular
// products): X reduced once to [0,2p); T = W Y in [0,2p) from W' = W beta mod p;
// X' = X + T, Y' = X - T + 2p in [0,4p).
template <class Wd>
__device__ __forceinline__ void bfly_inv_mont(typename Wd::T &x, typename Wd::T &y, typename Wd::T wm,
                                              typename Wd::T p, typename Wd::T p2, typename Wd::T j) {
  using T = typename Wd::T;
  const T xr = csub<T>(x, p2);
  const T t = mont_lazy<Wd>(y, wm, p, j);
  x = xr + t;
  y = xr - t + p2;
}

// Inverse butterfly with W = 1 in the lazy range: Y is brought to [0,2p) by
// one conditional subtraction instead of the product.
template <class Wd>
__device__ __forceinline__ void bfly_inv_lazy_w1(typename Wd::T &x, typename Wd::T &y, typename Wd::T p2) {
  using T = typename Wd::T;
  const T xr = csub<T>(x, p2);
  const T t = csub<T>(y, p2);
  x = xr + t;
  y = xr - t + p2;
}

// Plain inverse butterfly (X + W Y, X - W Y), X, Y in [0,p), every output fully reduced.
template <class Wd>
__device__ __forceinline__ void bfly_inv_plain(typename Wd::T &x, typename Wd::T &y, typename Wd::T w,
                                               typename Wd::T wp, typename Wd::T p) {
  using T = typename Wd::T;
  const T t = csub<T>(shoup_lazy_sub<Wd>(y, w, wp, p), p);
  const T s = csub<T>(x + t, p);
  T d = x - t;
  const T dp = d + p;
  y = dp < d ? dp : d;
  x = s;
}

template <class Wd>
__device__ __forceinline__ void bfly_inv_plain_w1(typename Wd::T &x, typename Wd::T &y, typename Wd::T p) {
  using T = typename Wd::T;
  const T s = csub<T>(x + y, p);
  T d = x - y;
  const T dp = d + p;
  y = dp < d ? dp : d;
  x = s;
}

}  // namespace hntt
