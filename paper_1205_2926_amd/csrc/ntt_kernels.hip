// Pass dispatch, the butterfly unit-test kernel and the pointwise product.
// The pass kernels themselves are in ntt_pass.hip.
//
// A transform of length L = 2^l is computed in at most two passes over HBM.
// Each pass stages a tile in LDS and runs several radix-2 stages of
// Algorithm 1 (Section 1) per LDS round trip: a thread loads 2^K elements
// whose indices differ in K adjacent bits, runs the K stages that pair those
// bits in registers, and writes them back.
//
//   kWhole  l <= 12: the whole transform in one workgroup.
//   kCols   the outer stages: L is viewed as an R x C row-major matrix
//           (R = 2^n rows, C columns).  Stages 1..n of Algorithm 1 only pair
//           elements of one column; they equal a length-R transform of each
//           column with root omega^C followed by the factor omega^(col*s) on
//           output s (the four-step split).  The factor comes from a table
//           laid out like the data.
//   kRows   the inner stages: each contiguous row of length C gets a
//           length-C transform with root omega^R.
// Forward: kCols then kRows (natural in, bit-reversed out).  Inverse: kRows
// then kCols, with the split factor conj(omega)^(col*s) * L^-1 applied on load.
#include "check_kernels.hpp"
#include "modarith.hpp"
#include "ntt_kernels.hpp"

namespace hntt {

namespace {

// ---------------------------------------------------------------------------------------------
template <class Wd>
__global__ void k_debug_butterfly(int kind, uint64_t p64, const typename Wd::T *x, const typename Wd::T *y,
                                  const typename Wd::T *w, const typename Wd::T *wp, typename Wd::T *xo,
                                  typename Wd::T *yo, size_t n) {
  using T = typename Wd::T;
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T p = (T)p64, p2 = p + p;
  T a = x[i], c = y[i];
  switch (kind) {
    case 0: bfly_fwd_plain<Wd>(a, c, w[i], wp[i], p); break;
    case 1: bfly_fwd_lazy<Wd>(a, c, w[i], wp[i], p, p2); break;
    case 2: bfly_inv_lazy<Wd>(a, c, w[i], wp[i], p, p2); break;
    case 4: bfly_fwd_mont<Wd>(a, c, w[i], p, p2, wp[i]); break;  // w = W beta mod p, wp = p^-1 mod beta
    case 5: bfly_inv_mont<Wd>(a, c, w[i], p, p2, wp[i]); break;
    default: bfly_inv_plain<Wd>(a, c, w[i], wp[i], p); break;
  }
  xo[i] = a;
  yo[i] = c;
}

// Montgomery product with beta = 2^bits (used only by the pointwise product,
// whose operands are both variable): for a, b < p < beta/4 returns
// a b beta^-1 mod p in [0,2p), in the form of Algorithm 5 with J = p^-1 mod beta.
template <class Wd>
__device__ __forceinline__ typename Wd::T mont_mul(typename Wd::T a, typename Wd::T b, typename Wd::T p,
                                                   typename Wd::T j) {
  using T = typename Wd::T;
  const T r1 = Wd::mulhi(a, b);
  const T r0 = Wd::mullo(a, b);
  const T q = Wd::mullo(r0, j);
  const T h = Wd::mulhi(q, p);
  return r1 - h + p;
}

template <class Wd>
__global__ void k_pointwise(uint64_t p64, uint64_t j64, uint64_t r2_64, const typename Wd::T *__restrict__ a,
                            const typename Wd::T *__restrict__ b, typename Wd::T *c, uint64_t len) {
  using T = typename Wd::T;
  const T p = (T)p64, j = (T)j64, r2 = (T)r2_64;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < len; i += (size_t)gridDim.x * blockDim.x) {
    T u = csub<T>(mont_mul<Wd>(a[i], b[i], p, j), p);  // a b / beta
    u = csub<T>(mont_mul<Wd>(u, r2, p, j), p);          // times beta^2 / beta
    c[i] = u;
  }
}

__global__ void k_set_flag(uint32_t *flag, uint32_t value) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = value;
}

// Lanes that saw an out-of-range word lower the flag with a vector atomic; the
// rest only read.
template <class T>
__global__ void k_range_check(const T *__restrict__ x, uint64_t len, T bound, uint32_t index, uint32_t *first_bad) {
  bool bad = false;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < len; i += (size_t)gridDim.x * blockDim.x)
    bad |= x[i] >= bound;
  if (bad) atomicMin(first_bad, index);
}

template <class T>
T inv_mod_pow2(T p) {  // p^-1 mod 2^bits for odd p, by Newton iteration
  T x = p;             // correct to 3 bits
  for (int i = 0; i < 6; ++i) x *= (T)2 - p * x;
  return x;
}

}  // namespace

size_t pass_lds_bytes(const PassParams &pp) {
  const RoundSplit sp = pass_split(pp.n, pp.word_bits, pp.kind == PassKind::kWhole);
  if (sp.kh == 0) return 0;
  const size_t wb = pp.word_bits / 8;
  const size_t N = (size_t)1 << pp.n;
  // per-stage twiddle table (N pairs) + padded tile (see LdsIO in ntt_pass.hip)
  const size_t padded = pp.kind == PassKind::kCols
                            ? N + N / 32
                            : row_padded_len(N) + row_skew(pp.n, sp.kh, sp.km, sp.kl, pp.word_bits);
  // (no LDS copy of the twiddle table where tw_global says so)
  const bool fwd = pp.kind != PassKind::kCols && !pp.inverse;
  const bool mem = tw_global(pp.n, pp.word_bits, fwd, pp.kind == PassKind::kWhole);
  const size_t bytes = wb * ((mem ? 0 : 2 * N) + padded * pp.group);
  return bytes <= 160 * 1024 ? bytes : 0;
}

hipError_t launch_pass(const PassParams &pp, const BatchPtrs &ptrs, hipStream_t stream) {
  if (pp.word_bits == 32) return pp.inverse ? launch_pass_u32_inv(pp, ptrs, stream) : launch_pass_u32_fwd(pp, ptrs, stream);
  return pp.inverse ? launch_pass_u64_inv(pp, ptrs, stream) : launch_pass_u64_fwd(pp, ptrs, stream);
}

hipError_t launch_debug_butterfly(int kind, int word_bits, uint64_t p, const void *x, const void *y, const void *w,
                                  const void *wp, void *xo, void *yo, size_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const int threads = 256;
  const int blocks = (int)((n + threads - 1) / threads);
  if (word_bits == 32) {
    using T = uint32_t;
    hipLaunchKernelGGL(k_debug_butterfly<Word32>, dim3(blocks), dim3(threads), 0, stream, kind, p,
                       (const T *)x, (const T *)y, (const T *)w, (const T *)wp, (T *)xo, (T *)yo, n);
  } else {
    using T = uint64_t;
    hipLaunchKernelGGL(k_debug_butterfly<Word64>, dim3(blocks), dim3(threads), 0, stream, kind, p,
                       (const T *)x, (const T *)y, (const T *)w, (const T *)wp, (T *)xo, (T *)yo, n);
  }
  return hipGetLastError();
}

hipError_t launch_set_flag(uint32_t *flag, uint32_t value, hipStream_t stream) {
  hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, stream, flag, value);
  return hipGetLastError();
}

hipError_t launch_range_check(int word_bits, const void *x, uint64_t len, uint64_t bound, uint32_t index,
                              uint32_t *first_bad, hipStream_t stream) {
  if (len == 0) return hipSuccess;
  const int threads = 256;
  const uint64_t want = (len + threads - 1) / threads;
  const int blocks = (int)(want < 4096 ? want : 4096);
  if (word_bits == 32)
    hipLaunchKernelGGL(k_range_check<uint32_t>, dim3(blocks), dim3(threads), 0, stream, (const uint32_t *)x, len,
                       (uint32_t)bound, index, first_bad);
  else
    hipLaunchKernelGGL(k_range_check<uint64_t>, dim3(blocks), dim3(threads), 0, stream, (const uint64_t *)x, len,
                       bound, index, first_bad);
  return hipGetLastError();
}

hipError_t launch_pointwise(int word_bits, uint64_t p, const void *a, const void *b, void *c, uint64_t len,
                            hipStream_t stream) {
  if (len == 0) return hipSuccess;
  const int threads = 256;
  const uint64_t want = (len + threads - 1) / threads;
  const int blocks = (int)(want < 8192 ? want : 8192);
  if (word_bits == 32) {
    using T = uint32_t;
    const T j = inv_mod_pow2<T>((T)p);
    const uint64_t beta_mod = (((uint64_t)1 << 32) % p);
    const uint64_t r2 = (uint64_t)(((unsigned __int128)beta_mod * beta_mod) % p);
    hipLaunchKernelGGL(k_pointwise<Word32>, dim3(blocks), dim3(threads), 0, stream, p, (uint64_t)j, r2,
                       (const T *)a, (const T *)b, (T *)c, len);
  } else {
    using T = uint64_t;
    const T j = inv_mod_pow2<T>(p);
    const unsigned __int128 beta = (unsigned __int128)1 << 64;
    const uint64_t beta_mod = (uint64_t)(beta % p);
    const uint64_t r2 = (uint64_t)(((unsigned __int128)beta_mod * beta_mod) % p);
    hipLaunchKernelGGL(k_pointwise<Word64>, dim3(blocks), dim3(threads), 0, stream, p, (uint64_t)j, r2,
                       (const T *)a, (const T *)b, (T *)c, len);
  }
  return hipGetLastError();
}

}  // namespace hntt
