// NTT pass kernels for gfx950.
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
#include "modarith.hpp"
#include "ntt_kernels.hpp"

namespace hntt {

namespace {

constexpr int kRadix = 4;  // stages per register round

// Element `pos` of sub-transform `g` in LDS.
struct RowLayout {
  int stride;
  __device__ __forceinline__ int operator()(int g, int pos) const { return g * stride + pos; }
};
struct ColLayout {
  int G;
  __device__ __forceinline__ int operator()(int g, int pos) const { return pos * G + g; }
};

template <class Wd, bool Lazy>
__device__ __forceinline__ void bfly_fwd(typename Wd::T &x, typename Wd::T &y, typename Wd::T w,
                                         typename Wd::T wp, typename Wd::T p, typename Wd::T p2) {
  if constexpr (Lazy) bfly_fwd_lazy<Wd>(x, y, w, wp, p, p2);
  else bfly_fwd_plain<Wd>(x, y, w, wp, p);
}
template <class Wd, bool Lazy>
__device__ __forceinline__ void bfly_fwd_w1(typename Wd::T &x, typename Wd::T &y, typename Wd::T p,
                                            typename Wd::T p2) {
  if constexpr (Lazy) bfly_fwd_lazy_w1<Wd>(x, y, p2);
  else bfly_fwd_plain_w1<Wd>(x, y, p);
}
template <class Wd, bool Lazy>
__device__ __forceinline__ void bfly_inv(typename Wd::T &x, typename Wd::T &y, typename Wd::T w,
                                         typename Wd::T wp, typename Wd::T p, typename Wd::T p2) {
  if constexpr (Lazy) bfly_inv_lazy<Wd>(x, y, w, wp, p, p2);
  else bfly_inv_plain<Wd>(x, y, w, wp, p);
}
template <class Wd, bool Lazy>
__device__ __forceinline__ void bfly_inv_w1(typename Wd::T &x, typename Wd::T &y, typename Wd::T p,
                                            typename Wd::T p2) {
  if constexpr (Lazy) bfly_inv_lazy_w1<Wd>(x, y, p2);
  else bfly_inv_plain_w1<Wd>(x, y, p);
}

// One register round of K forward (DIF) stages on the bits [b_lo, b_lo + K) of
// the position.  Stage i of Algorithm 1 pairs bit b = n - i with twiddle
// zeta_i^(pos mod 2^b) = omega_N^((pos mod 2^b) << (i - 1)).
template <class Wd, bool Lazy, int K, class Layout>
__device__ __forceinline__ void fwd_round(typename Wd::T *lds, Layout lay, int n, int b_lo, int g, int t, int tpt,
                                          const typename Wd::T *tw, const typename Wd::T *twp, typename Wd::T p,
                                          typename Wd::T p2) {
  using T = typename Wd::T;
  const int groups = 1 << (n - K);
  for (int gi = t; gi < groups; gi += tpt) {
    const int low = gi & ((1 << b_lo) - 1);
    const int base = ((gi >> b_lo) << (b_lo + K)) | low;
    T v[1 << K];
#pragma unroll
    for (int e = 0; e < (1 << K); ++e) v[e] = lds[lay(g, base | (e << b_lo))];
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const int hb = K - 1 - s;
      const int b = b_lo + hb;
      if (b == 0) {
#pragma unroll
        for (int e = 0; e < (1 << K); ++e)
          if (!(e & (1 << hb))) bfly_fwd_w1<Wd, Lazy>(v[e], v[e | (1 << hb)], p, p2);
      } else {
        const int shift = n - 1 - b;
#pragma unroll
        for (int e = 0; e < (1 << K); ++e)
          if (!(e & (1 << hb))) {
            const int pos = base | (e << b_lo);
            const int idx = (pos & ((1 << b) - 1)) << shift;
            bfly_fwd<Wd, Lazy>(v[e], v[e | (1 << hb)], tw[idx], twp[idx], p, p2);
          }
      }
    }
#pragma unroll
    for (int e = 0; e < (1 << K); ++e) lds[lay(g, base | (e << b_lo))] = v[e];
  }
}

// One register round of K inverse stages (Algorithm 1 run backwards): bits
// b_lo upward, butterfly (X + W Y, X - W Y) with W = omega_N^(-(pos mod 2^b) << (i-1)).
template <class Wd, bool Lazy, int K, class Layout>
__device__ __forceinline__ void inv_round(typename Wd::T *lds, Layout lay, int n, int b_lo, int g, int t, int tpt,
                                          const typename Wd::T *tw, const typename Wd::T *twp, typename Wd::T p,
                                          typename Wd::T p2) {
  using T = typename Wd::T;
  const int groups = 1 << (n - K);
  for (int gi = t; gi < groups; gi += tpt) {
    const int low = gi & ((1 << b_lo) - 1);
    const int base = ((gi >> b_lo) << (b_lo + K)) | low;
    T v[1 << K];
#pragma unroll
    for (int e = 0; e < (1 << K); ++e) v[e] = lds[lay(g, base | (e << b_lo))];
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const int hb = s;
      const int b = b_lo + hb;
      if (b == 0) {
#pragma unroll
        for (int e = 0; e < (1 << K); ++e)
          if (!(e & (1 << hb))) bfly_inv_w1<Wd, Lazy>(v[e], v[e | (1 << hb)], p, p2);
      } else {
        const int shift = n - 1 - b;
#pragma unroll
        for (int e = 0; e < (1 << K); ++e)
          if (!(e & (1 << hb))) {
            const int pos = base | (e << b_lo);
            const int idx = (pos & ((1 << b) - 1)) << shift;
            bfly_inv<Wd, Lazy>(v[e], v[e | (1 << hb)], tw[idx], twp[idx], p, p2);
          }
      }
    }
#pragma unroll
    for (int e = 0; e < (1 << K); ++e) lds[lay(g, base | (e << b_lo))] = v[e];
  }
}

// All n stages of a length-2^n sub-transform held in LDS.  Rounds of kRadix
// stages; the remainder round takes the innermost bits.
template <class Wd, bool Lazy, bool Inverse, class Layout>
__device__ void sub_transform(typename Wd::T *lds, Layout lay, int n, int g, int t, int tpt, const typename Wd::T *tw,
                              const typename Wd::T *twp, typename Wd::T p) {
  using T = typename Wd::T;
  const T p2 = p + p;
  const int nr = (n + kRadix - 1) / kRadix;
  const int rem = n - kRadix * (nr - 1);
  for (int r = 0; r < nr; ++r) {
    // forward: round r covers bits [n - 4(r+1), n - 4r) except the last (rem bits at 0);
    // inverse: the same rounds in reverse order.
    const int rr = Inverse ? (nr - 1 - r) : r;
    const bool last = (rr == nr - 1);
    const int b_lo = last ? 0 : n - kRadix * (rr + 1);
    const int k = last ? rem : kRadix;
    if constexpr (Inverse) {
      switch (k) {
        case 1: inv_round<Wd, Lazy, 1>(lds, lay, n, b_lo, g, t, tpt, tw, twp, p, p2); break;
        case 2: inv_round<Wd, Lazy, 2>(lds, lay, n, b_lo, g, t, tpt, tw, twp, p, p2); break;
        case 3: inv_round<Wd, Lazy, 3>(lds, lay, n, b_lo, g, t, tpt, tw, twp, p, p2); break;
        default: inv_round<Wd, Lazy, 4>(lds, lay, n, b_lo, g, t, tpt, tw, twp, p, p2); break;
      }
    } else {
      switch (k) {
        case 1: fwd_round<Wd, Lazy, 1>(lds, lay, n, b_lo, g, t, tpt, tw, twp, p, p2); break;
        case 2: fwd_round<Wd, Lazy, 2>(lds, lay, n, b_lo, g, t, tpt, tw, twp, p, p2); break;
        case 3: fwd_round<Wd, Lazy, 3>(lds, lay, n, b_lo, g, t, tpt, tw, twp, p, p2); break;
        default: fwd_round<Wd, Lazy, 4>(lds, lay, n, b_lo, g, t, tpt, tw, twp, p, p2); break;
      }
    }
    __syncthreads();
  }
}

template <class T>
__device__ __forceinline__ void stage_table(T *dst_w, T *dst_wp, const T *src_w, const T *src_wp, int count) {
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    dst_w[i] = src_w[i];
    dst_wp[i] = src_wp[i];
  }
}

// Final reduction of a lazy result: forward outputs lie in [0,2p), inverse in [0,4p).
template <class Wd, bool Lazy, bool Inverse>
__device__ __forceinline__ typename Wd::T normalize(typename Wd::T x, typename Wd::T p) {
  using T = typename Wd::T;
  if constexpr (!Lazy) return x;
  if constexpr (Inverse) x = csub<T>(x, p + p);
  return csub<T>(x, p);
}

// ---------------------------------------------------------------------------------------------
// kWhole and kRows: each workgroup owns `group` contiguous rows of length 2^n
// (kWhole: one whole transform per row, log_other = 0).
template <class Wd, bool Lazy, bool Inverse>
__global__ void __launch_bounds__(1024) k_rows(BatchPtrs ptrs, int n, int log_rows, int group, uint64_t p64,
                                               const typename Wd::T *__restrict__ tw_g,
                                               const typename Wd::T *__restrict__ twp_g, int normalize_out,
                                               uint64_t scale_w64, uint64_t scale_wp64) {
  using T = typename Wd::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const T p = (T)p64;
  const int N = 1 << n;
  const int half = N >> 1;
  T *tw = reinterpret_cast<T *>(smem_raw);
  T *twp = tw + half;
  T *data = twp + half;

  const int groups_per_transform = (1 << log_rows) / group;
  const int b = blockIdx.x / groups_per_transform;
  const int rg = blockIdx.x % groups_per_transform;
  T *gdata = reinterpret_cast<T *>(ptrs.ptr[b]) + ((size_t)rg * group << n);

  stage_table<T>(tw, twp, tw_g, twp_g, half);
  const int total = group << n;
  for (int i = threadIdx.x; i < total; i += blockDim.x) data[i] = gdata[i];
  __syncthreads();

  const int tpt = blockDim.x / group;
  const int g = threadIdx.x / tpt;
  const int t = threadIdx.x % tpt;
  sub_transform<Wd, Lazy, Inverse>(data, RowLayout{N}, n, g, t, tpt, tw, twp, p);

  const bool scale = Inverse && log_rows == 0;  // whole inverse transform: times L^-1
  const T sw = (T)scale_w64, swp = (T)scale_wp64;
  for (int i = threadIdx.x; i < total; i += blockDim.x) {
    T x = data[i];
    if (scale) {
      x = shoup_lazy<Wd>(x, sw, swp, p);  // any x < beta -> [0,2p)
      x = csub<T>(x, p);
    } else if (normalize_out) {
      x = normalize<Wd, Lazy, Inverse>(x, p);
    }
    gdata[i] = x;
  }
}

// kCols: each workgroup owns `group` adjacent columns of the R x C view
// (R = 2^n rows, C = 2^log_cols columns).
template <class Wd, bool Lazy, bool Inverse>
__global__ void __launch_bounds__(1024) k_cols(BatchPtrs ptrs, int n, int log_cols, int group, uint64_t p64,
                                               const typename Wd::T *__restrict__ tw_g,
                                               const typename Wd::T *__restrict__ twp_g,
                                               const typename Wd::T *__restrict__ tt_w,
                                               const typename Wd::T *__restrict__ tt_wp, int normalize_out) {
  using T = typename Wd::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const T p = (T)p64;
  const int R = 1 << n;
  const int half = R >> 1;
  const size_t C = (size_t)1 << log_cols;
  T *tw = reinterpret_cast<T *>(smem_raw);
  T *twp = tw + half;
  T *data = twp + half;

  const int groups_per_transform = (int)(C / group);
  const int b = blockIdx.x / groups_per_transform;
  const int c0 = (blockIdx.x % groups_per_transform) * group;
  T *gdata = reinterpret_cast<T *>(ptrs.ptr[b]);

  stage_table<T>(tw, twp, tw_g, twp_g, half);
  const int total = group << n;
  for (int i = threadIdx.x; i < total; i += blockDim.x) {
    const int row = i / group, col = i % group;
    const size_t gi = (size_t)row * C + c0 + col;
    T x = gdata[gi];
    if constexpr (Inverse) {
      // split twiddle conj(omega)^(col*s) * L^-1 before the column transform
      x = shoup_lazy<Wd>(x, tt_w[gi], tt_wp[gi], p);
      if constexpr (!Lazy) x = csub<T>(x, p);
    }
    data[i] = x;
  }
  __syncthreads();

  const int tpt = blockDim.x / group;
  const int g = threadIdx.x % group;
  const int t = threadIdx.x / group;
  sub_transform<Wd, Lazy, Inverse>(data, ColLayout{group}, n, g, t, tpt, tw, twp, p);

  for (int i = threadIdx.x; i < total; i += blockDim.x) {
    const int row = i / group, col = i % group;
    const size_t gi = (size_t)row * C + c0 + col;
    T x = data[i];
    if constexpr (!Inverse) {
      // split twiddle omega^(col*s) after the column transform
      x = shoup_lazy<Wd>(x, tt_w[gi], tt_wp[gi], p);
      if constexpr (!Lazy) x = csub<T>(x, p);
    } else if (normalize_out) {
      x = normalize<Wd, Lazy, true>(x, p);
    }
    gdata[gi] = x;
  }
}

template <class Wd, bool Lazy, bool Inverse>
hipError_t launch_typed(const PassParams &pp, const BatchPtrs &ptrs, hipStream_t stream) {
  using T = typename Wd::T;
  const int tpt = pp.n > kRadix ? (1 << (pp.n - kRadix)) : 1;
  const int threads = tpt * pp.group;
  const size_t lds = pass_lds_bytes(pp);
  if (threads > 1024 || lds == 0) return hipErrorInvalidValue;
  const T *tw = static_cast<const T *>(pp.tw_w);
  const T *twp = static_cast<const T *>(pp.tw_wp);
  static bool attr_set = false;  // allow the full 160 KiB of LDS once per instantiation
  if (!attr_set) {
    hipFuncSetAttribute(reinterpret_cast<const void *>(&k_cols<Wd, Lazy, Inverse>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    hipFuncSetAttribute(reinterpret_cast<const void *>(&k_rows<Wd, Lazy, Inverse>),
                        hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr_set = true;
  }
  if (pp.kind == PassKind::kCols) {
    const int blocks = ((1 << pp.log_other) / pp.group) * pp.nbatch;
    hipLaunchKernelGGL((k_cols<Wd, Lazy, Inverse>), dim3(blocks), dim3(threads), lds, stream, ptrs, pp.n,
                       pp.log_other, pp.group, pp.p, tw, twp, static_cast<const T *>(pp.tt_w),
                       static_cast<const T *>(pp.tt_wp), (int)pp.normalize);
  } else {
    const int log_rows = pp.kind == PassKind::kWhole ? 0 : pp.log_other;
    const int blocks = ((1 << log_rows) / pp.group) * pp.nbatch;
    hipLaunchKernelGGL((k_rows<Wd, Lazy, Inverse>), dim3(blocks), dim3(threads), lds, stream, ptrs, pp.n, log_rows,
                       pp.group, pp.p, tw, twp, (int)pp.normalize, pp.scale_w, pp.scale_wp);
  }
  return hipGetLastError();
}

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

template <class T>
T inv_mod_pow2(T p) {  // p^-1 mod 2^bits for odd p, by Newton iteration
  T x = p;             // correct to 3 bits
  for (int i = 0; i < 6; ++i) x *= (T)2 - p * x;
  return x;
}

}  // namespace

size_t pass_lds_bytes(const PassParams &pp) {
  const size_t wb = pp.word_bits / 8;
  const size_t N = (size_t)1 << pp.n;
  const size_t bytes = wb * (N + N * pp.group);  // twiddle table (N/2 pairs) + tile
  return bytes <= 160 * 1024 ? bytes : 0;
}

hipError_t launch_pass(const PassParams &pp, const BatchPtrs &ptrs, hipStream_t stream) {
  if (pp.word_bits == 32) {
    if (pp.lazy) return pp.inverse ? launch_typed<Word32, true, true>(pp, ptrs, stream)
                                   : launch_typed<Word32, true, false>(pp, ptrs, stream);
    return pp.inverse ? launch_typed<Word32, false, true>(pp, ptrs, stream)
                      : launch_typed<Word32, false, false>(pp, ptrs, stream);
  }
  if (pp.lazy) return pp.inverse ? launch_typed<Word64, true, true>(pp, ptrs, stream)
                                 : launch_typed<Word64, true, false>(pp, ptrs, stream);
  return pp.inverse ? launch_typed<Word64, false, true>(pp, ptrs, stream)
                    : launch_typed<Word64, false, false>(pp, ptrs, stream);
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
