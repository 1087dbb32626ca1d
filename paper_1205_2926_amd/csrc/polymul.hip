// Kernels of the three-prime polynomial product (the application named in
// Section 1 of the paper): operand preparation, the pointwise product of the
// transforms, and Chinese remaindering of the three residue vectors (Garner).
// All three are persistent: a fixed grid of workgroups strides over a table of
// 1024-word chunks covering every product of the batch.
#include "modarith.hpp"
#include "polymul_kernels.hpp"

namespace hntt {
namespace {

constexpr int kChunk = 1024;
constexpr int kThreads = 256;

// x mod q for any 32-bit x: Shoup product by 1 (W' = floor(2^32 / q)) then one correction.
__device__ __forceinline__ uint32_t reduce_u32(uint32_t x, uint32_t q, uint32_t one_p) {
  return csub<uint32_t>(shoup_lazy<Word32>(x, 1u, one_p, q), q);
}

// c * x mod q, fully reduced, for a constant c with Shoup constant cp.
__device__ __forceinline__ uint32_t mulc(uint32_t x, uint32_t c, uint32_t cp, uint32_t q) {
  return csub<uint32_t>(shoup_lazy<Word32>(x, c, cp, q), q);
}

__device__ __forceinline__ uint32_t subm(uint32_t a, uint32_t b, uint32_t q) {
  const uint32_t d = a - b;
  const uint32_t dq = d + q;
  return dq < d ? dq : d;  // a >= b: d < q <= dq (no wrap) ; a < b: d wraps, dq = a - b + q < q
}

// Montgomery product a b 2^-32 mod q in [0, 2q) for a, b < 2q, q < 2^30 (the form of Algorithm 5).
__device__ __forceinline__ uint32_t mont(uint32_t a, uint32_t b, uint32_t q, uint32_t j) {
  const uint32_t r1 = __umulhi(a, b);
  const uint32_t r0 = a * b;
  const uint32_t m = r0 * j;
  const uint32_t h = __umulhi(m, q);
  return r1 - h + q;
}

__global__ void __launch_bounds__(kThreads) k_poly_prep(PolyArgs args) {
  for (int c = blockIdx.x; c < args.nchunks_ws; c += gridDim.x) {
    const ChunkEntry ce = args.chunks_ws[c];
    const PolyPair pp = args.pairs[ce.pair];
    const uint32_t L = 1u << pp.log2_len;
    uint32_t *ws = args.workspace + pp.ws_off;
    for (uint32_t j = ce.start + threadIdx.x; j < ce.start + kChunk && j < L; j += kThreads) {
      const uint32_t av = j < pp.na ? pp.a[j] : 0u;
      const uint32_t bv = j < pp.nb ? pp.b[j] : 0u;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const PrimeConst &pc = args.primes[k];
        ws[(2 * k) * (size_t)L + j] = reduce_u32(av, pc.q, pc.one_p);
        ws[(2 * k + 1) * (size_t)L + j] = reduce_u32(bv, pc.q, pc.one_p);
      }
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_poly_pointwise(PolyArgs args) {
  for (int c = blockIdx.x; c < args.nchunks_ws; c += gridDim.x) {
    const ChunkEntry ce = args.chunks_ws[c];
    const PolyPair pp = args.pairs[ce.pair];
    const uint32_t L = 1u << pp.log2_len;
    uint32_t *ws = args.workspace + pp.ws_off;
    for (uint32_t j = ce.start + threadIdx.x; j < ce.start + kChunk && j < L; j += kThreads) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const PrimeConst &pc = args.primes[k];
        uint32_t *A = ws + (2 * k) * (size_t)L;
        const uint32_t *B = ws + (2 * k + 1) * (size_t)L;
        uint32_t u = csub<uint32_t>(mont(A[j], B[j], pc.q, pc.jinv), pc.q);  // a b 2^-32
        A[j] = csub<uint32_t>(mont(u, pc.r2, pc.q, pc.jinv), pc.q);          // times 2^64 2^-32
      }
    }
  }
}

// Garner: v1 = r1, v2 = (r2 - v1) q1^-1 mod q2, v3 = ((r3 - v1) q1^-1 - v2) q2^-1 mod q3,
// x = v1 + q1 (v2 + q2 v3) mod 2^64.
__global__ void __launch_bounds__(kThreads) k_poly_crt(PolyArgs args) {
  const PrimeConst &P1 = args.primes[0], &P2 = args.primes[1], &P3 = args.primes[2];
  const CrtConst cc = args.crt;
  for (int c = blockIdx.x; c < args.nchunks_out; c += gridDim.x) {
    const ChunkEntry ce = args.chunks_out[c];
    const PolyPair pp = args.pairs[ce.pair];
    const uint32_t L = 1u << pp.log2_len;
    const uint32_t nout = pp.na + pp.nb - 1;
    const uint32_t *ws = args.workspace + pp.ws_off;
    for (uint32_t j = ce.start + threadIdx.x; j < ce.start + kChunk && j < nout; j += kThreads) {
      const uint32_t r1 = ws[j], r2 = ws[2 * (size_t)L + j], r3 = ws[4 * (size_t)L + j];
      const uint32_t v1 = r1;
      const uint32_t v2 = mulc(subm(r2, reduce_u32(v1, P2.q, P2.one_p), P2.q), cc.c12, cc.c12p, P2.q);
      uint32_t t = mulc(subm(r3, reduce_u32(v1, P3.q, P3.one_p), P3.q), cc.c13, cc.c13p, P3.q);
      t = subm(t, reduce_u32(v2, P3.q, P3.one_p), P3.q);
      const uint32_t v3 = mulc(t, cc.c23, cc.c23p, P3.q);
      pp.out[j] = (uint64_t)v1 + (uint64_t)P1.q * ((uint64_t)v2 + (uint64_t)P2.q * v3);
    }
  }
}

int grid_for(int chunks) {
  const int cap = 256 * 8;  // 8 workgroups per CU on 256 CUs
  return chunks < cap ? (chunks > 0 ? chunks : 1) : cap;
}

}  // namespace

hipError_t launch_poly_prep(const PolyArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_poly_prep, dim3(grid_for(a.nchunks_ws)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_poly_pointwise(const PolyArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_poly_pointwise, dim3(grid_for(a.nchunks_ws)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_poly_crt(const PolyArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_poly_crt, dim3(grid_for(a.nchunks_out)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace hntt
