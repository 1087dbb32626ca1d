// Kernels of the three-prime polynomial product (the application named in
// Section 1 of the paper): operand preparation and Chinese remaindering of the
// three residue vectors (Garner), plus the carry pass of large-integer
// products.  (The pointwise product of the transforms is fused into the last
// forward pass of the B_k.)  All are persistent: a fixed grid of workgroups
// strides over a table of 1024-word chunks covering every product of the batch.
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

__global__ void __launch_bounds__(kThreads) k_poly_prep(PolyArgs args) {
  for (int c = blockIdx.x; c < args.nchunks_ws; c += gridDim.x) {
    const ChunkEntry ce = args.chunks_ws[c];
    const PolyPair pp = args.pairs[ce.pair];
    const uint32_t L = 1u << pp.log2_len;
    uint32_t *ws = args.workspace + pp.ws_off;
    // the lower half only: na, nb <= L / 2, and the first forward pass reads the
    // upper half as zero without loading it.  A is stored times beta = 2^32 mod q,
    // so that the pointwise product fused into the B transforms' last pass is one
    // Montgomery product (B A beta beta^-1 = A B).
    for (uint32_t j = ce.start + threadIdx.x; j < ce.start + kChunk && j < L / 2; j += kThreads) {
      const uint32_t av = j < pp.na ? pp.a[j] : 0u;
      const uint32_t bv = j < pp.nb ? pp.b[j] : 0u;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const PrimeConst &pc = args.primes[k];
        ws[(2 * k) * (size_t)L + j] = mulc(av, pc.beta, pc.beta_p, pc.q);
        ws[(2 * k + 1) * (size_t)L + j] = reduce_u32(bv, pc.q, pc.one_p);
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
      static_cast<uint64_t *>(pp.out)[j] = (uint64_t)v1 + (uint64_t)P1.q * ((uint64_t)v2 + (uint64_t)P2.q * v3);
    }
  }
}

// Garner as above, but the coefficient x = v1 + q1 v2 + q1 q2 v3 < 2^89 is kept
// whole: its three 32-bit words go to B1[j], B2[j], B3[j] (free once the B_k
// transforms have multiplied into the A_k).  Exact for any 32-bit limbs: x <= min(na, nb) (2^32 - 1)^2
// < 2^86 < q1 q2 q3 when min(na, nb) <= 2^22.
// The three 32-bit words of coefficient j of a product (its residues are at ws[j],
// ws[2L + j], ws[4L + j]).
__device__ __forceinline__ void garner_words(const PolyArgs &args, const uint32_t *ws, uint32_t L, uint32_t j,
                                             uint32_t &w0, uint32_t &w1, uint32_t &w2) {
  const PrimeConst &P1 = args.primes[0], &P2 = args.primes[1], &P3 = args.primes[2];
  const CrtConst &cc = args.crt;
  const uint32_t r1 = ws[j], r2 = ws[2 * (size_t)L + j], r3 = ws[4 * (size_t)L + j];
  const uint32_t v1 = r1;
  const uint32_t v2 = mulc(subm(r2, reduce_u32(v1, P2.q, P2.one_p), P2.q), cc.c12, cc.c12p, P2.q);
  uint32_t t = mulc(subm(r3, reduce_u32(v1, P3.q, P3.one_p), P3.q), cc.c13, cc.c13p, P3.q);
  t = subm(t, reduce_u32(v2, P3.q, P3.one_p), P3.q);
  const uint32_t v3 = mulc(t, cc.c23, cc.c23p, P3.q);
  // 128-bit sum: a = v1 + q1 v2 < 2^61; q12 v3 from the 32-bit halves of q12 (< 2^60)
  const uint64_t q12 = args.q12;
  const uint64_t a = (uint64_t)v1 + (uint64_t)P1.q * v2;
  const uint64_t p0 = (uint64_t)(uint32_t)q12 * v3;
  const uint64_t p1 = (q12 >> 32) * v3;
  const uint64_t lo = p0 + (p1 << 32);
  uint64_t hi = (p1 >> 32) + (lo < p0 ? 1 : 0);
  const uint64_t lo2 = lo + a;
  hi += lo2 < lo ? 1 : 0;
  w0 = (uint32_t)lo2;
  w1 = (uint32_t)(lo2 >> 32);
  w2 = (uint32_t)hi;
}

// Carry pass.  With the coefficient words w0, w1, w2 of c_j (c_j = w0 + w1 2^32 +
// w2 2^64), the product is sum_k s_k 2^(32k) with s_k = w0[k] + w1[k-1] + w2[k-2]
// < 3 2^32.  Write s_k = lo_k + 2^32 hi_k (hi_k <= 2) and t_k = lo_k + hi_(k-1)
// <= 2^32 + 1; then limb k is (t_k + c_k) mod 2^32 with carry c_(k+1) =
// (t_k + c_k) >> 32 in {0, 1} and c_0 = 0.  Each position is a carry state:
// generate (t_k >= 2^32: carry out 1), propagate (t_k = 2^32 - 1: carry out =
// carry in) or kill (carry out 0).  A run of positions composes to its rightmost
// non-propagate state, so the carries are an associative scan: per chunk, then
// per product over its chunks, then inside each chunk again.
enum : uint32_t { kKill = 0, kGen = 1, kProp = 2 };

constexpr int kPerThread = kChunk / kThreads;  // consecutive limbs per thread
static_assert(kPerThread == 4, "a thread's limbs are stored as one 16-byte vector");

// The three words of the exact coefficients of one product (written over B_1, B_2,
// B_3) and its lengths: s_k = w0[k] + w1[k-1] + w2[k-2] for k < nlimb.
struct BigView {
  const uint32_t *w0, *w1, *w2;
  uint32_t nout, nlimb;
};

__device__ __forceinline__ BigView big_view(const PolyArgs &args, const PolyPair &pp) {
  const uint32_t L = 1u << pp.log2_len;
  const uint32_t *ws = args.workspace + pp.ws_off;
  return BigView{ws + (size_t)L, ws + 3 * (size_t)L, ws + 5 * (size_t)L, pp.na + pp.nb - 1, pp.na + pp.nb};
}

__device__ __forceinline__ uint32_t fold(uint32_t left, uint32_t right) { return right == kProp ? left : right; }

// Carry into each thread of a 256-thread workgroup given the states of the
// threads (in order) and the carry `cin` into thread 0; also returns the
// workgroup's composed state in *all.  Uses wave ballots: the carry into a lane
// is set by the nearest lane below it whose state is not propagate.
__device__ __forceinline__ uint32_t wg_carry_in(uint32_t state, uint32_t cin, uint32_t *lds, uint32_t *all) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t nonp = __ballot(state != kProp);
  const uint64_t gen = __ballot(state == kGen);
  if (lane == 0) lds[wave] = nonp ? (uint32_t)((gen >> (63 - __clzll(nonp))) & 1) : kProp;
  __syncthreads();
  uint32_t c = cin;
  for (int w = 0; w < wave; ++w) c = fold(c, lds[w]);
  uint32_t a = kProp;
  for (int w = 0; w < kThreads / 64; ++w) a = fold(a, lds[w]);
  const uint64_t below = nonp & ((1ull << lane) - 1);
  if (below) c = (uint32_t)((gen >> (63 - __clzll(below))) & 1);
  __syncthreads();  // lds is reused by the caller's next scan
  *all = a;
  return c;
}

// Garner for the coefficients of one 1024-limb chunk, written to B1, B2, B3 as
// above, and, from the same words kept in LDS (plus the three coefficients before
// the chunk, recomputed), the chunk's composed carry state.
__global__ void __launch_bounds__(kThreads) k_big_crt_state(PolyArgs args) {
  constexpr int kHalo = 3;  // s_(k-1) for the chunk's first limb needs coefficient start - 3
  __shared__ uint32_t W[3][kChunk + kHalo];
  __shared__ uint32_t lds[kThreads / 64];
  for (int c = blockIdx.x; c < args.nchunks_out; c += gridDim.x) {
    const ChunkEntry ce = args.chunks_out[c];
    const PolyPair pp = args.pairs[ce.pair];
    const uint32_t L = 1u << pp.log2_len;
    const uint32_t nout = pp.na + pp.nb - 1, nlimb = pp.na + pp.nb;
    uint32_t *ws = args.workspace + pp.ws_off;
    const int64_t j0 = (int64_t)ce.start - kHalo;  // coefficient of LDS entry 0
    for (int i = threadIdx.x; i < kChunk + kHalo; i += kThreads) {
      const int64_t j = j0 + i;
      uint32_t w0 = 0, w1 = 0, w2 = 0;
      if (j >= 0 && j < (int64_t)nout) {
        garner_words(args, ws, L, (uint32_t)j, w0, w1, w2);
        if (i >= kHalo) {  // this chunk's own coefficients
          ws[1 * (size_t)L + j] = w0;
          ws[3 * (size_t)L + j] = w1;
          ws[5 * (size_t)L + j] = w2;
        }
      }
      W[0][i] = w0;
      W[1][i] = w1;
      W[2][i] = w2;
    }
    __syncthreads();
    // s_k = w0[k] + w1[k-1] + w2[k-2] from LDS (zero outside the product)
    auto s_at = [&](int64_t k) -> uint64_t {
      if (k < 0 || k >= (int64_t)nlimb) return 0;
      const int i = (int)(k - j0);
      return (uint64_t)W[0][i] + W[1][i - 1] + W[2][i - 2];
    };
    const int64_t k0 = (int64_t)ce.start + threadIdx.x * kPerThread;
    uint64_t prev = s_at(k0 - 1);
    uint32_t mine = kProp;
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
      const uint64_t cur = s_at(k0 + i);
      const uint64_t t = (cur & 0xFFFFFFFFull) + (prev >> 32);
      const uint32_t st = (k0 + i >= (int64_t)nlimb) ? kProp
                          : t >= (1ull << 32)          ? kGen
                          : t == 0xFFFFFFFFull         ? kProp
                                                       : kKill;
      mine = fold(mine, st);
      prev = cur;
    }
    uint32_t all;
    (void)wg_carry_in(mine, 0, lds, &all);  // ends with a barrier: W may be reused
    if (threadIdx.x == 0) args.chunk_state[c] = all;
  }
}

// One workgroup per product: the carry into each of its chunks.
__global__ void __launch_bounds__(kThreads) k_big_chunk_carry(PolyArgs args) {
  __shared__ uint32_t lds[kThreads / 64];
  for (int i = blockIdx.x; i < args.npairs; i += gridDim.x) {
    const PolyPair pp = args.pairs[i];
    const uint32_t nchunks = (pp.na + pp.nb + kChunk - 1) / kChunk;
    const uint32_t per = (nchunks + kThreads - 1) / kThreads;
    const uint32_t c0 = pp.chunk0 + threadIdx.x * per;
    const uint32_t c1 = min(pp.chunk0 + nchunks, c0 + per);
    uint32_t mine = kProp;
    for (uint32_t c = c0; c < c1; ++c) mine = fold(mine, args.chunk_state[c]);
    uint32_t all;
    uint32_t carry = wg_carry_in(mine, 0, lds, &all);
    for (uint32_t c = c0; c < c1; ++c) {
      args.chunk_carry[c] = carry;
      carry = fold(carry, args.chunk_state[c]);
    }
  }
}

// The chunk's words are first copied into LDS with coalesced loads (each thread's
// four consecutive limbs would otherwise read every word four lanes apart), and
// each thread stores its four limbs as one 16-byte vector.
__global__ void __launch_bounds__(kThreads) k_big_apply(PolyArgs args) {
  constexpr int kHalo = 3;
  __shared__ uint32_t W[3][kChunk + kHalo];
  __shared__ uint32_t lds[kThreads / 64];
  for (int c = blockIdx.x; c < args.nchunks_out; c += gridDim.x) {
    const ChunkEntry ce = args.chunks_out[c];
    const PolyPair pp = args.pairs[ce.pair];
    const BigView v = big_view(args, pp);
    const int64_t j0 = (int64_t)ce.start - kHalo;  // coefficient of LDS entry 0
    for (int i = threadIdx.x; i < kChunk + kHalo; i += kThreads) {
      const int64_t j = j0 + i;
      const bool in = j >= 0 && j < (int64_t)v.nout;
      W[0][i] = in ? v.w0[j] : 0u;
      W[1][i] = in ? v.w1[j] : 0u;
      W[2][i] = in ? v.w2[j] : 0u;
    }
    __syncthreads();
    auto s_at = [&](int64_t k) -> uint64_t {  // s_k from LDS, 0 outside the product
      if (k < 0 || k >= (int64_t)v.nlimb) return 0;
      const int i = (int)(k - j0);
      return (uint64_t)W[0][i] + W[1][i - 1] + W[2][i - 2];
    };
    const int64_t k0 = (int64_t)ce.start + threadIdx.x * kPerThread;
    uint64_t t[kPerThread];
    uint32_t mine = kProp;
    uint64_t prev = s_at(k0 - 1);
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
      const uint64_t cur = s_at(k0 + i);
      t[i] = (cur & 0xFFFFFFFFull) + (prev >> 32);
      const uint32_t st = (k0 + i >= (int64_t)v.nlimb) ? kProp
                          : t[i] >= (1ull << 32)       ? kGen
                          : t[i] == 0xFFFFFFFFull      ? kProp
                                                       : kKill;
      mine = fold(mine, st);
      prev = cur;
    }
    uint32_t all;
    uint32_t carry = wg_carry_in(mine, args.chunk_carry[c], lds, &all);  // ends with a barrier
    uint32_t o[kPerThread];
#pragma unroll
    for (int i = 0; i < kPerThread; ++i) {
      const uint64_t x = t[i] + carry;
      o[i] = (uint32_t)x;
      carry = (uint32_t)(x >> 32);
    }
    uint32_t *out = static_cast<uint32_t *>(pp.out) + k0;
    if (k0 + kPerThread <= (int64_t)v.nlimb && (reinterpret_cast<uintptr_t>(out) & 15) == 0) {
      *reinterpret_cast<uint4 *>(out) = make_uint4(o[0], o[1], o[2], o[3]);
    } else {
#pragma unroll
      for (int i = 0; i < kPerThread; ++i)
        if (k0 + i < (int64_t)v.nlimb) out[i] = o[i];
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
hipError_t launch_poly_crt(const PolyArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_poly_crt, dim3(grid_for(a.nchunks_out)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_big_crt(const PolyArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_big_crt_state, dim3(grid_for(a.nchunks_out)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_big_carry(const PolyArgs &a, hipStream_t s) {
  hipError_t e;
  hipLaunchKernelGGL(k_big_chunk_carry, dim3(grid_for(a.npairs)), dim3(kThreads), 0, s, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_big_apply, dim3(grid_for(a.nchunks_out)), dim3(kThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace hntt
