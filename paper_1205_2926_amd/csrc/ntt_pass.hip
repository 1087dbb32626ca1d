// One NTT pass kernel family, compiled once per (word size, direction):
// HNTT_WORD = 32 | 64, HNTT_INVERSE = 0 | 1, and templated on the butterfly
// policy (Algorithm 2, Algorithms 3/4, or Algorithm 5 and its inverse), the pass
// kind and the register rounds.
//
// A workgroup owns G sub-transforms of length N = 2^n (n = KH + KM + KL):
//   rows  G contiguous rows of a transform viewed as (#rows x N)   (also whole
//         transforms: one row, #rows = 1)
//   cols  G adjacent columns of a transform viewed as (N x #cols), row-major.
// The n radix-2 stages of Algorithm 1 (Section 1) run in up to three register
// rounds: the "high" round pairs position bits [KM + KL, n), the middle round
// bits [KL, KL + KM) and the "low" round bits [0, KL).  A thread keeps the 2^K
// elements of one group in registers for all K stages of a round, and the tile
// crosses LDS between rounds:
//   forward (DIF):  HBM -> high -> LDS -> (middle -> LDS ->) low -> HBM
//   inverse (DIT):  HBM -> low -> LDS -> (middle -> LDS ->) high -> HBM
// With KH = 0 there is one round and no LDS tile.  Global loads and stores are
// issued directly by the rounds that touch HBM; lanes are laid out so that each
// memory instruction covers contiguous words (columns fastest in a cols pass,
// positions fastest in a rows pass).  The forward row pass writes its output
// through LDS so that consecutive lanes store consecutive 16 bytes, and when a
// row has fewer than 32 threads it also reads its input through LDS.  Every
// thread issues all of its loads for such an LDS copy before the first wait.
//
// Twiddles of the high and middle rounds depend on the thread's low position
// bits and are read from an LDS copy of the table; twiddles of the low round
// are uniform across the workgroup (their indices are compile-time multiples of
// 2^(n-1-b)), so they come straight from global memory through scalar loads,
// and the butterflies whose twiddle is 1 skip the product entirely.  The split
// twiddle of a two-pass transform is applied where the data enters the second
// pass (Edge), and the final forward pass of a polynomial product can multiply
// its output into a partner transform (the pointwise product, GlobalIO::pm).
#include <type_traits>

#include "modarith.hpp"
#include "ntt_kernels.hpp"

#ifndef HNTT_WORD
#error "HNTT_WORD must be 32 or 64"
#endif
#ifndef HNTT_INVERSE
#error "HNTT_INVERSE must be 0 or 1"
#endif

#if HNTT_WORD == 32 && HNTT_INVERSE == 0
#define HNTT_NS pass_u32_fwd
#elif HNTT_WORD == 32
#define HNTT_NS pass_u32_inv
#elif HNTT_INVERSE == 0
#define HNTT_NS pass_u64_fwd
#else
#define HNTT_NS pass_u64_inv
#endif

namespace hntt {
namespace HNTT_NS {

#if HNTT_WORD == 32
using Wd = Word32;
#else
using Wd = Word64;
#endif
using T = typename Wd::T;
constexpr bool kInverse = HNTT_INVERSE != 0;
// Sub-transforms whose high and middle rounds read their twiddles from global
// memory (L1/L2) instead of an LDS copy (tw_global in ntt_kernels.hpp).
constexpr bool tw_global_here(int n) { return tw_global(n, HNTT_WORD); }

// Global (HBM) address space: lets the compiler emit global_* instead of flat_*
// memory instructions, which would also count against the LDS wait counter.
#define HNTT_GLOBAL __attribute__((address_space(1)))

// A twiddle W and its Shoup constant W' as one 2-word vector (.x = W, .y = W').
typedef T Tw2 __attribute__((ext_vector_type(2)));
// 16 bytes moved by one vector memory instruction.
typedef uint32_t Vec16 __attribute__((ext_vector_type(4)));

// Raw buffer accesses: 32-bit per-lane byte offset + uniform byte offset on a
// buffer resource (base, size); accesses beyond the size read 0 / are dropped.
constexpr int kBufferFlags = 0x00020000;  // gfx9 family raw-buffer descriptor word 3
// A workgroup-uniform 64-bit value, marked uniform for the compiler (it must be
// uniform already: this reads lane 0's copy).
__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (uint64_t)lo | ((uint64_t)hi << 32);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kBufferFlags);
}
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(T) == 4) {
    return (T)__builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
  } else {
    typedef int V2 __attribute__((ext_vector_type(2)));
    const V2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
    return (T)(uint32_t)v.x | ((T)(uint32_t)v.y << 32);
  }
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, T x) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32((int)x, r, (int)voff, (int)soff, 0);
  } else {
    typedef int V2 __attribute__((ext_vector_type(2)));
    V2 v;
    v.x = (int)(uint32_t)x;
    v.y = (int)(uint32_t)(x >> 32);
    __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)voff, (int)soff, 0);
  }
}
// Twiddle table entry of a policy: (W, W') pair for Shoup products, the single
// word W beta mod p for Montgomery products.
template <int Pol>
struct TwOf {
  using type = Tw2;
};
template <>
struct TwOf<kPolicyMont> {
  using type = T;
};
template <int Pol>
using TwT = typename TwOf<Pol>::type;

template <int Pol>
__device__ __forceinline__ TwT<Pol> buf_load_tw(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  if constexpr (Pol == kPolicyMont) {
    return buf_load(r, voff, soff);
  } else {
    Tw2 w;
    if constexpr (sizeof(T) == 4) {
      typedef int V2 __attribute__((ext_vector_type(2)));
      const V2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
      w.x = (T)(uint32_t)v.x;
      w.y = (T)(uint32_t)v.y;
    } else {
      typedef int V4 __attribute__((ext_vector_type(4)));
      const V4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
      w.x = (T)(uint32_t)v.x | ((T)(uint32_t)v.y << 32);
      w.y = (T)(uint32_t)v.z | ((T)(uint32_t)v.w << 32);
    }
    return w;
  }
}

// The modulus of a launch: p, 2p and (Montgomery policy) p^-1 mod beta.
struct Mod {
  T p, p2, j;
};

template <int Pol>
__device__ __forceinline__ void bfly(T &x, T &y, const TwT<Pol> &tw, const Mod &m) {
  if constexpr (Pol == kPolicyMont) {
    if constexpr (kInverse) bfly_inv_mont<Wd>(x, y, tw, m.p, m.p2, m.j);
    else bfly_fwd_mont<Wd>(x, y, tw, m.p, m.p2, m.j);
  } else if constexpr (kInverse) {
    if constexpr (Pol == kPolicyLazy) bfly_inv_lazy<Wd>(x, y, tw.x, tw.y, m.p, m.p2);
    else bfly_inv_plain<Wd>(x, y, tw.x, tw.y, m.p);
  } else {
    if constexpr (Pol == kPolicyLazy) bfly_fwd_lazy<Wd>(x, y, tw.x, tw.y, m.p, m.p2);
    else bfly_fwd_plain<Wd>(x, y, tw.x, tw.y, m.p);
  }
}

// Butterfly whose twiddle is 1: no product (both lazy policies share the ranges).
template <int Pol>
__device__ __forceinline__ void bfly_w1(T &x, T &y, const Mod &m) {
  if constexpr (kInverse) {
    if constexpr (Pol != kPolicyPlain) bfly_inv_lazy_w1<Wd>(x, y, m.p2);
    else bfly_inv_plain_w1<Wd>(x, y, m.p);
  } else {
    if constexpr (Pol != kPolicyPlain) bfly_fwd_lazy_w1<Wd>(x, y, m.p2);
    else bfly_fwd_plain_w1<Wd>(x, y, m.p);
  }
}

// x (any word) times a table constant, result in [0,2p).
template <int Pol>
__device__ __forceinline__ T mul_const(T x, const TwT<Pol> &tw, const Mod &m) {
  if constexpr (Pol == kPolicyMont) return mont_lazy<Wd>(x, tw, m.p, m.j);
  else if constexpr (!kInverse) return shoup_lazy_mad<Wd>(x, tw.x, tw.y, m.p);
  else return shoup_lazy<Wd>(x, tw.x, tw.y, m.p);
}

// Words per 16-byte vector access.
constexpr int kVec = 16 / sizeof(T);

// One round of K stages on the position bits [b_lo, b_lo + K).  Stage i of
// Algorithm 1 pairs bit b = n - i; its twiddle is zeta_i^(pos mod 2^b), which is
// entry (1 << b) + (pos mod 2^b) of the per-stage ("heap") table, so that lanes
// with consecutive positions read consecutive entries.
// LowRound: b_lo = 0, the twiddle indices are compile-time constants and are
// read from global memory with scalar loads; the butterflies with twiddle 1
// skip the product.  Otherwise the twiddles come from the LDS copy `tws`.
// Src/Dst provide load2/store2 of one position given as a per-lane part plus a
// uniform part with disjoint bits, and load_vec/store_vec of kVec consecutive
// positions when their kContig flag is set.
// after_load runs once per thread, after the loads of its first group are issued
// and before the stages (the twiddle staging below uses it to overlap the two).
// ZU (first round of a forward transform only, where the round's top bit is the
// position's top bit): words of the upper half read as 0 without being loaded.
// A template parameter, so that rounds without it compile exactly as before.
struct NoHook {
  __device__ __forceinline__ void operator()() const {}
};

template <int Pol, int N_LOG, int K, bool LowRound, bool ZU = false, class Src, class Dst, class Hook = NoHook>
__device__ __forceinline__ void round_k(int b_lo, int t, int tpt, const TwT<Pol> *tws,
                                       const HNTT_GLOBAL TwT<Pol> *__restrict__ twg, const Mod &m, const Src &src,
                                       const Dst &dst, const Hook &after_load = Hook{}) {
  constexpr int groups = 1 << (N_LOG - K);
  constexpr int M = 1 << K;
#pragma unroll 1
  for (int gi = t; gi < groups; gi += tpt) {
    const int low = gi & ((1 << b_lo) - 1);
    const int base = ((gi >> b_lo) << (b_lo + K)) | low;
    T v[M];
    if constexpr (LowRound && Src::kContig && M >= kVec) {
#pragma unroll
      for (int e = 0; e < M; e += kVec) {
        if (ZU && ((e >> (K - 1)) & 1)) {  // the whole vector lies in the upper half
#pragma unroll
          for (int i = 0; i < kVec; ++i) v[e + i] = 0;
        } else {
          src.load_vec(base + e, &v[e]);
          if constexpr (ZU) {
#pragma unroll
            for (int i = 0; i < kVec; ++i)
              if (((e + i) >> (K - 1)) & 1) v[e + i] = 0;
          }
        }
      }
    } else {
#pragma unroll
      for (int e = 0; e < M; ++e) v[e] = (ZU && ((e >> (K - 1)) & 1)) ? (T)0 : src.load2(base, e << b_lo);
    }
    // Every thread runs groups / tpt >= 1 iterations, so a hook that synchronises
    // the workgroup is reached once by all threads.
    if (gi == t) {
      after_load();
      if constexpr (kInverse) __builtin_amdgcn_s_setprio(0);  // raised at the start of k_pass
    }
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const int hb = kInverse ? s : K - 1 - s;
#pragma unroll
      for (int e = 0; e < M; ++e) {
        if (e & (1 << hb)) continue;
        if constexpr (LowRound) {
          const int kk = e & ((1 << hb) - 1);
          if (kk == 0) {
            bfly_w1<Pol>(v[e], v[e | (1 << hb)], m);
          } else {
            const TwT<Pol> tw = twg[(1 << hb) + kk];
            bfly<Pol>(v[e], v[e | (1 << hb)], tw, m);
          }
        } else {
          const int b = b_lo + hb;
          const int pos = base | (e << b_lo);
          const int ti = (1 << b) + (pos & ((1 << b) - 1));
          const TwT<Pol> tw = tw_global_here(N_LOG) ? twg[ti] : tws[ti];
          bfly<Pol>(v[e], v[e | (1 << hb)], tw, m);
        }
      }
    }
    if constexpr (LowRound && Dst::kContig && M >= kVec) {
#pragma unroll
      for (int e = 0; e < M; e += kVec) dst.store_vec(base + e, &v[e]);
    } else {
#pragma unroll
      for (int e = 0; e < M; ++e) dst.store2(base, e << b_lo, v[e]);
    }
  }
}

// Final reduction of a lazy result: forward outputs lie in [0,2p), inverse in [0,4p).
template <int Pol>
__device__ __forceinline__ T reduce_final(T x, T p) {
  if constexpr (Pol == kPolicyPlain) return x;
  if constexpr (kInverse) x = csub<T>(x, p + p);
  return csub<T>(x, p);
}

struct KernelArgs {
  BatchPtrs ptrs;             // transforms (slot 0) when `table` is null
  const XformEntry *table;    // else: device table of (pointer, prime slot)
  int units;                  // tiles per transform (the grid is units x transforms)
  int log_other;              // rows: log2(#rows); cols: log2(#columns)
  int group;                  // G
  int normalize;              // reduce the final output to [0,p)
  int scale;                  // whole inverse: multiply by L^-1 (slot scale_w, scale_wp)
  uint32_t pm_off;            // fused pointwise product into the partner transform (0: off)
  int zero_upper;             // first forward pass: the upper half of every input is zero, not read
  SlotParams slots[kMaxSlots];
};

// The fused pointwise product of a final forward pass: a b mod p for a, b in [0,p),
// as two Montgomery products (a b beta^-1, then times beta^2 beta^-1), fully reduced.
__device__ __forceinline__ T pmul_word(T a, T b, const Mod &m, T r2) {
  const T u = csub<T>(mont_lazy<Wd>(a, b, m.p, m.j), m.p);
  return csub<T>(mont_lazy<Wd>(u, r2, m.p, m.j), m.p);
}

// What happens to a word on its way in from HBM and out to HBM.  The split
// twiddle of a two-pass transform is applied where the data enters the second
// pass: on load in the row pass (forward: omega^(s pos) for row s's position
// pos) and on load in the column pass (inverse: L^-1 conj(omega)^(col rev(pos))).
// It is the product of two factors, one indexed by the low SIGMA bits of the
// position and one by the remaining high bits, read from a per-sub-transform
// table [low factors (2^SIGMA pairs) | high factors (2^(n-SIGMA) pairs)] that is
// small enough to stay in the L1/L2 caches.  SIGMA is the bit boundary of the
// pass's first register round, so one factor is fixed per thread group and the
// other is shared by all lanes of a sub-transform.  TT = false: no split twiddle.
// Out fixes what out() does: kOutRaw passes words through (the first pass of a
// two-pass transform), kOutNorm reduces them to [0,p), kOutCond reduces them
// with p replaced by 0 when normalisation is off (the same instructions either
// way, no select), kOutAny follows the runtime flags (whole inverse transforms,
// which may also scale by L^-1).  The final round of a pass picks its variant
// with one uniform branch: with the flags tested per word, the compiler computes
// the reduction for every word and selects afterwards, also when it is not wanted.
constexpr int kOutRaw = 0, kOutNorm = 1, kOutAny = 2, kOutCond = 3;
template <int Pol, bool Cols, bool TT, int N_LOG, int SIGMA, int Out = kOutAny>
struct Edge {
  Mod m;
  int normalize, scale;
  T sw, swp;
  __amdgpu_buffer_rsrc_t tt;  // factor tables of the pass
  uint32_t tt_off;            // byte offset of this sub-transform's first factor
  uint32_t tt_step;           // bytes between consecutive factors of one sub-transform
  // pos = lp + up with disjoint bits: lp varies per lane, up is uniform
  __device__ __forceinline__ T in(T x, int lp, int up) const {
    if constexpr (TT) {
      constexpr int kMask = (1 << SIGMA) - 1;
      const TwT<Pol> hi = buf_load_tw<Pol>(tt, tt_off + (uint32_t)((1 << SIGMA) + (lp >> SIGMA)) * tt_step,
                                           (uint32_t)(up >> SIGMA) * tt_step);
      const TwT<Pol> lo = buf_load_tw<Pol>(tt, tt_off + (uint32_t)(lp & kMask) * tt_step,
                                           (uint32_t)(up & kMask) * tt_step);
      x = mul_const<Pol>(x, hi, m);  // any input < beta -> [0,2p)
      x = mul_const<Pol>(x, lo, m);
      if constexpr (Pol == kPolicyPlain) x = csub<T>(x, m.p);
    }
    return x;
  }
  __device__ __forceinline__ T in(T x, int pos) const { return in(x, pos, 0); }
  template <int O>
  __device__ __forceinline__ Edge<Pol, Cols, TT, N_LOG, SIGMA, O> with_out() const {
    return {m, normalize, scale, sw, swp, tt, tt_off, tt_step};
  }
  __device__ __forceinline__ T out(T x, int pos) const {
    if constexpr (Out == kOutRaw) {
      return x;
    } else if constexpr (Out == kOutNorm) {
      return reduce_final<Pol>(x, m.p);
    } else if constexpr (Out == kOutCond) {
      return reduce_final<Pol>(x, normalize ? m.p : (T)0);
    } else if constexpr (!Cols && kInverse) {
      if (scale) {  // whole inverse transform: times L^-1, then reduced
        if constexpr (Pol == kPolicyMont) x = mont_lazy<Wd>(x, sw, m.p, m.j);
        else x = shoup_lazy<Wd>(x, sw, swp, m.p);
        if (normalize) x = csub<T>(x, m.p);
      } else if (normalize) {
        x = reduce_final<Pol>(x, m.p);
      }
    } else {
      if (normalize) x = reduce_final<Pol>(x, m.p);
    }
    return x;
  }
};

// HBM side: position pos of this thread's sub-transform is word off + pos*stride
// of the transform at `base`.  The base is uniform across the workgroup (scalar
// registers) and the offset is 32-bit, so accesses use the scalar-base addressing
// form instead of per-lane 64-bit address arithmetic.
template <bool Cols, class EdgeT>
struct GlobalIO {
  static constexpr bool kContig = !Cols;
  HNTT_GLOBAL T *base;
  HNTT_GLOBAL T *pm;            // rows/whole forward: partner base of the fused product, or null
  T r2;
  __amdgpu_buffer_rsrc_t rsrc;  // Cols: the transform as a buffer
  uint32_t off;
  uint32_t stride;
  EdgeT edge;
  // the same view with another output variant of the edge
  template <int O>
  __device__ __forceinline__ auto with_out() const {
    GlobalIO<Cols, decltype(edge.template with_out<O>())> g;
    g.base = base;
    g.pm = pm;
    g.r2 = r2;
    g.rsrc = rsrc;
    g.off = off;
    g.stride = stride;
    g.edge = edge.template with_out<O>();
    return g;
  }
  __device__ __forceinline__ T load2(int lp, int up) const {
    if constexpr (Cols) {
      const T x = buf_load(rsrc, (off + (uint32_t)lp * stride) * (uint32_t)sizeof(T),
                           (uint32_t)up * stride * (uint32_t)sizeof(T));
      return edge.in(x, lp, up);
    } else {
      return edge.in(base[off + (uint32_t)(lp + up)], lp, up);
    }
  }
  __device__ __forceinline__ void store2(int lp, int up, T x) const {
    x = edge.out(x, lp + up);
    if constexpr (!Cols && !kInverse) {  // (the fused product ends forward transforms only)
      if (pm) {
        HNTT_GLOBAL T *q = pm + off + (uint32_t)(lp + up);
        *q = pmul_word(x, *q, edge.m, r2);
        return;
      }
    }
    if constexpr (Cols) {
      buf_store(rsrc, (off + (uint32_t)lp * stride) * (uint32_t)sizeof(T), (uint32_t)up * stride * (uint32_t)sizeof(T),
                x);
    } else {
      base[off + (uint32_t)(lp + up)] = x;
    }
  }
  // kContig only: kVec consecutive positions, pos a multiple of kVec
  __device__ __forceinline__ void load_vec(int pos, T *v) const {
    const Vec16 q = *reinterpret_cast<const HNTT_GLOBAL Vec16 *>(base + (off + (uint32_t)pos));
    const T *w = reinterpret_cast<const T *>(&q);
#pragma unroll
    for (int i = 0; i < kVec; ++i) v[i] = edge.in(w[i], pos + i);
  }
  __device__ __forceinline__ void store_vec(int pos, const T *v) const {
    Vec16 q;
    T *w = reinterpret_cast<T *>(&q);
#pragma unroll
    for (int i = 0; i < kVec; ++i) w[i] = edge.out(v[i], pos + i);
    if (!kInverse && pm) {
      HNTT_GLOBAL Vec16 *dst = reinterpret_cast<HNTT_GLOBAL Vec16 *>(pm + (off + (uint32_t)pos));
      const Vec16 pa = *dst;
      const T *pw = reinterpret_cast<const T *>(&pa);
#pragma unroll
      for (int i = 0; i < kVec; ++i) w[i] = pmul_word(w[i], pw[i], edge.m, r2);
      *dst = q;
      return;
    }
    *reinterpret_cast<HNTT_GLOBAL Vec16 *>(base + (off + (uint32_t)pos)) = q;
  }
};

// LDS side.  Columns: element (g, pos) at pad1(pos) * G + g, one pad word per 32
// positions, so both rounds' access patterns hit distinct banks.  Rows: element
// (g, pos) at g * pitch + pos + 4 (pos >> 5) (row_padded_len), which keeps the
// 16-byte alignment of vector accesses.
template <bool Cols>
struct LdsIO {
  static constexpr bool kContig = !Cols;
  T *tile;
  int G, g, pitch;
  __device__ __forceinline__ int idx(int pos) const {
    if constexpr (Cols) return (pos + (pos >> 5)) * G + g;
    else return g * pitch + pos + ((pos >> 5) << 2);
  }
  __device__ __forceinline__ T load2(int lp, int up) const { return tile[idx(lp + up)]; }
  __device__ __forceinline__ void store2(int lp, int up, T x) const { tile[idx(lp + up)] = x; }
  __device__ __forceinline__ void load_vec(int pos, T *v) const {
    const Vec16 q = *reinterpret_cast<const Vec16 *>(tile + idx(pos));
    const T *w = reinterpret_cast<const T *>(&q);
#pragma unroll
    for (int i = 0; i < kVec; ++i) v[i] = w[i];
  }
  __device__ __forceinline__ void store_vec(int pos, const T *v) const {
    Vec16 q;
    T *w = reinterpret_cast<T *>(&q);
#pragma unroll
    for (int i = 0; i < kVec; ++i) w[i] = v[i];
    *reinterpret_cast<Vec16 *>(tile + idx(pos)) = q;
  }
};

// An LDS tile read as the input of a pass: words go through the pass's input
// edge (the split twiddle) as they leave LDS.
template <class EdgeT>
struct LdsEdgeIO {
  static constexpr bool kContig = true;
  LdsIO<false> lio;
  EdgeT edge;
  __device__ __forceinline__ T load2(int lp, int up) const { return edge.in(lio.load2(lp, up), lp, up); }
  __device__ __forceinline__ void load_vec(int pos, T *v) const {
    lio.load_vec(pos, v);
#pragma unroll
    for (int i = 0; i < kVec; ++i) v[i] = edge.in(v[i], pos + i);
  }
};

// Copy of the N-entry heap twiddle table into LDS, in two steps so that its global
// loads are in flight together with the tile's: load() issues up to kR loads per
// thread into registers, store() writes them to LDS (and copies any remainder).
template <int Pol, int N>
struct TwStage {
  static constexpr int N_LOG2 = __builtin_ctz(N);
  static constexpr int kR = 8;
  TwT<Pol> r[kR];
  int nthr;  // threads in the workgroup
  __device__ __forceinline__ void load(const HNTT_GLOBAL TwT<Pol> *__restrict__ twg) {
    if constexpr (tw_global_here(N_LOG2)) return;
#pragma unroll
    for (int j = 0; j < kR; ++j) {
      const int i = threadIdx.x + j * nthr;
      if (i < N) r[j] = twg[i];
    }
  }
  __device__ __forceinline__ void store(TwT<Pol> *tws, const HNTT_GLOBAL TwT<Pol> *__restrict__ twg) const {
    if constexpr (tw_global_here(N_LOG2)) return;
#pragma unroll
    for (int j = 0; j < kR; ++j) {
      const int i = threadIdx.x + j * nthr;
      if (i < N) tws[i] = r[j];
    }
    for (int i = threadIdx.x + kR * nthr; i < N; i += nthr) tws[i] = twg[i];
  }
};

// Padded LDS words per sub-transform (rows: row pitch; cols: rows of the tile).
template <bool Cols>
constexpr int padded_len(int N) {
  return Cols ? N + N / 32 : (int)row_padded_len((size_t)N);
}

template <int Pol, bool Cols, int KH, int KM, int KL, bool TT>
__global__ void __launch_bounds__(kMaxPassThreads) k_pass(KernelArgs a) {
  constexpr int N_LOG = KH + KM + KL;
  // bit boundary of the first register round (split-twiddle factorisation)
  constexpr int SIGMA = kInverse ? KL : (KM + KL);
  constexpr int N = 1 << N_LOG;
  constexpr int KMAX = KH > KL ? (KH > KM ? KH : KM) : (KL > KM ? KL : KM);
  constexpr int TPT = 1 << (N_LOG - KMAX);
  static_assert(KH > 0 || KM == 0, "a single round has no middle round");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // Inverse passes: a wave keeps a raised issue priority until its first group's
  // loads (and the split-twiddle products applied to them) are issued, so that a
  // starting workgroup's memory requests go out ahead of the arithmetic of the
  // workgroup it shares the CU with (the inverse column pass ran 9% faster; the
  // forward passes, whose loads are followed by the twiddle staging, ran slower).
  if constexpr (kInverse) __builtin_amdgcn_s_setprio(3);
  const int units = a.units;
  const int G = a.group;
  int g, t;
  if constexpr (Cols) {
    g = threadIdx.x % G;
    t = threadIdx.x / G;
  } else {
    t = threadIdx.x % TPT;
    g = threadIdx.x / TPT;
  }
  const size_t C = (size_t)1 << a.log_other;
  TwT<Pol> *tws = reinterpret_cast<TwT<Pol> *>(smem_raw);
  T *tile = tw_global_here(N_LOG) ? reinterpret_cast<T *>(smem_raw) : reinterpret_cast<T *>(tws + N);

  // One tile (transform b, unit) per workgroup.  Blocks are dealt to the 8 XCDs
  // round-robin; each XCD takes a contiguous eighth of the units for every transform,
  // units fastest: neighbouring column groups (which share 128-byte lines) then run
  // together in one L2, and an XCD re-reads only its own eighth of the split twiddles.
  {
    const int tl = blockIdx.x;
    int b, unit;
    if ((units & 7) == 0) {
      const int x = tl & 7, j = tl >> 3, per = units >> 3;
      unit = x * per + j % per;
      b = j / per;
    } else {
      unit = tl % units;
      b = tl / units;
    }
    int slot = 0;
    uint64_t ptr;
    if (a.table) {
      ptr = a.table[b].ptr;
      slot = (int)a.table[b].slot;
    } else {
      ptr = a.ptrs.ptr[b];
    }
    // select the slot with uniform branches (indexing the kernel-argument array with
    // a runtime value would copy it to scratch memory)
    SlotParams sp = a.slots[0];
    if (slot == 1) sp = a.slots[1];
    else if (slot == 2) sp = a.slots[2];
    else if (slot == 3) sp = a.slots[3];
    const T p = (T)sp.p;
    const Mod m{p, p + p, (T)sp.jinv};
    const HNTT_GLOBAL TwT<Pol> *__restrict__ twg = (const HNTT_GLOBAL TwT<Pol> *)(sp.tw);

    HNTT_GLOBAL T *const gbase = (HNTT_GLOBAL T *)(uniform64(ptr));
    using EdgeT = Edge<Pol, Cols, TT, N_LOG, SIGMA>;
    EdgeT edge{m, a.normalize, a.scale, (T)sp.scale_w, (T)sp.scale_wp, make_rsrc(sp.tt, 0), 0, 0};
    GlobalIO<Cols, EdgeT> gio;
    constexpr uint32_t kTw = sizeof(TwT<Pol>);
    constexpr uint32_t kTTStride = (1u << SIGMA) + (1u << (N_LOG - SIGMA));
    const uint32_t nsub = Cols ? (uint32_t)C : (1u << a.log_other);  // sub-transforms per transform
    if constexpr (TT)
      edge.tt = make_rsrc((const void *)uniform64((uint64_t)sp.tt), nsub * kTTStride * kTw);
    gio.base = gbase;
    gio.pm = a.pm_off ? gbase - a.pm_off : nullptr;
    gio.r2 = (T)sp.r2;
    if constexpr (Cols) {
      const uint32_t col = (uint32_t)unit * G + g;
      gio.rsrc = make_rsrc((const void *)gbase, (uint32_t)(C * N * sizeof(T)));
      gio.off = col;
      gio.stride = (uint32_t)C;
      // factor-major table [factor][column]: adjacent columns' factors are adjacent
      edge.tt_off = col * kTw;
      edge.tt_step = (uint32_t)C * kTw;
    } else {
      const uint32_t row = (uint32_t)unit * G + g;
      gio.off = row * N;
      gio.stride = 1;
      // row-major table [row][factor]: a row's lanes read consecutive low factors
      edge.tt_off = row * kTTStride * kTw;
      edge.tt_step = kTw;
    }
    gio.edge = edge;

    if constexpr (KH == 0) {
      // one round, HBM to HBM
      if (!kInverse && a.zero_upper) round_k<Pol, N_LOG, KL, true, true>(0, t, TPT, nullptr, twg, m, gio, gio);
      else round_k<Pol, N_LOG, KL, true>(0, t, TPT, nullptr, twg, m, gio, gio);
    } else {
      // The twiddle table's loads are issued first and written to LDS only after
      // the tile's loads are in flight: one memory round trip before the stages.
      const int nthr = G * TPT;  // blockDim.x
      TwStage<Pol, N> stage;
      stage.nthr = nthr;
      stage.load(twg);
      const LdsIO<Cols> lio{tile, G, g, padded_len<Cols>(N)};
      if constexpr (!kInverse) {
        // Rows with fewer than 32 threads per row: a high-round load instruction would
        // cover under 128 bytes of each row, so the tile is first copied into LDS with
        // consecutive lanes on consecutive 16 bytes, and the high round reads it there.
        constexpr bool kCopyIn = !Cols && TPT < 32;
        if constexpr (kCopyIn) {
          constexpr int kPitch = padded_len<false>(N);
          constexpr int kChunks = N / kVec;
          constexpr int kPer = kChunks / TPT;  // vectors per thread
          static_assert(kPer * TPT == kChunks && kPer % 2 == 0, "copy-in covers the tile exactly");
          const HNTT_GLOBAL T *const rows0 = gbase + (size_t)unit * G * N;
          // ZU: only the lower half of each row is copied, and the high round reads
          // the upper half as zero (a compile-time choice: no per-lane branch between
          // a load and its use).
          const auto copy_in = [&](auto zu_tag) {
            constexpr bool ZU = decltype(zu_tag)::value;
            constexpr int kCh = ZU ? kChunks / 2 : kChunks;  // chunks read per row
            constexpr int kLoad = ZU ? kPer / 2 : kPer;
            Vec16 q[kLoad];
#pragma unroll
            for (int j = 0; j < kLoad; ++j) {
              const int i = threadIdx.x + j * nthr;
              q[j] = *reinterpret_cast<const HNTT_GLOBAL Vec16 *>(rows0 + (size_t)(i / kCh) * N + (i % kCh) * kVec);
            }
#pragma unroll
            for (int j = 0; j < kLoad; ++j) {
              const int i = threadIdx.x + j * nthr;
              const int row = i / kCh, c = (i % kCh) * kVec;
              *reinterpret_cast<Vec16 *>(tile + row * kPitch + c + ((c >> 5) << 2)) = q[j];
            }
            stage.store(tws, twg);
            __syncthreads();  // tile and twiddle table staged
            const LdsEdgeIO<EdgeT> lin{lio, edge};
            round_k<Pol, N_LOG, KH, false, ZU>(KM + KL, t, TPT, tws, twg, m, lin, lio);
          };
          if (a.zero_upper) copy_in(std::true_type{});
          else copy_in(std::false_type{});
        } else if constexpr (TT) {
          // the split twiddle's products follow the loads and would all have to
          // finish before a barrier placed after them: the table goes first
          stage.store(tws, twg);
          __syncthreads();  // twiddle table staged
          if (a.zero_upper) round_k<Pol, N_LOG, KH, false, true>(KM + KL, t, TPT, tws, twg, m, gio, lio);
          else round_k<Pol, N_LOG, KH, false>(KM + KL, t, TPT, tws, twg, m, gio, lio);
        } else {
          const auto staged = [&]() {
            stage.store(tws, twg);
            __syncthreads();  // twiddle table staged
          };
          if (a.zero_upper) round_k<Pol, N_LOG, KH, false, true>(KM + KL, t, TPT, tws, twg, m, gio, lio, staged);
          else round_k<Pol, N_LOG, KH, false>(KM + KL, t, TPT, tws, twg, m, gio, lio, staged);
        }
        __syncthreads();
        if constexpr (KM > 0) {
          round_k<Pol, N_LOG, KM, false>(KL, t, TPT, tws, twg, m, lio, lio);
          __syncthreads();
        }
        if constexpr (Cols) {
          // the forward column pass is always the first of two: its output is never
          // reduced (the launcher rejects the flag)
          round_k<Pol, N_LOG, KL, true>(0, t, TPT, tws, twg, m, lio, gio.template with_out<kOutRaw>());
        } else {
          // Rows: a thread's low-round outputs are 2^KL consecutive words, so direct
          // stores would put neighbouring lanes 2^KL words apart.  Stage them in LDS
          // and write the tile out with consecutive lanes on consecutive 16 bytes.
          round_k<Pol, N_LOG, KL, true>(0, t, TPT, tws, twg, m, lio, lio);
          __syncthreads();
          // (every thread moves kPer vectors; the partner words of the fused product
          // are all requested before the first is used)
          constexpr int kPitch = padded_len<false>(N);
          constexpr int kChunks = N / kVec;
          constexpr int kPer = kChunks / TPT;
          static_assert(kPer * TPT == kChunks, "copy-out covers the tile exactly");
          const size_t tile0 = (size_t)unit * G * N;
          const auto ed = edge.template with_out<kOutCond>();
          Vec16 o[kPer];
#pragma unroll
          for (int j = 0; j < kPer; ++j) {
            const int i = threadIdx.x + j * nthr;
            const int row = i / kChunks, c = (i % kChunks) * kVec;
            const Vec16 q = *reinterpret_cast<const Vec16 *>(tile + row * kPitch + c + ((c >> 5) << 2));
            const T *w = reinterpret_cast<const T *>(&q);
            T *wo = reinterpret_cast<T *>(&o[j]);
#pragma unroll
            for (int e = 0; e < kVec; ++e) wo[e] = ed.out(w[e], c + e);
          }
          HNTT_GLOBAL T *const out0 = (gio.pm ? gio.pm : gbase) + tile0;
          if (gio.pm) {  // fused pointwise product into the partner transform
            Vec16 pa[kPer];
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
              const int i = threadIdx.x + j * nthr;
              pa[j] = *reinterpret_cast<const HNTT_GLOBAL Vec16 *>(out0 + (size_t)(i / kChunks) * N +
                                                                    (i % kChunks) * kVec);
            }
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
              const T *pw = reinterpret_cast<const T *>(&pa[j]);
              T *wo = reinterpret_cast<T *>(&o[j]);
#pragma unroll
              for (int e = 0; e < kVec; ++e) wo[e] = pmul_word(wo[e], pw[e], m, gio.r2);
            }
          }
#pragma unroll
          for (int j = 0; j < kPer; ++j) {
            const int i = threadIdx.x + j * nthr;
            *reinterpret_cast<HNTT_GLOBAL Vec16 *>(out0 + (size_t)(i / kChunks) * N + (i % kChunks) * kVec) = o[j];
          }
        }
      } else {
        // With the split twiddle the table is written first: keeping its registers
        // live through the round costs the round's loads their overlap.
        if constexpr (TT) stage.store(tws, twg);
        round_k<Pol, N_LOG, KL, true>(0, t, TPT, tws, twg, m, gio, lio);
        if constexpr (!TT) stage.store(tws, twg);
        __syncthreads();  // tile and twiddle table complete
        if constexpr (KM > 0) {
          round_k<Pol, N_LOG, KM, false>(KL, t, TPT, tws, twg, m, lio, lio);
          __syncthreads();
        }
        const auto last = [&](const auto &dst) {
          round_k<Pol, N_LOG, KH, false>(KM + KL, t, TPT, tws, twg, m, lio, dst);
        };
        if constexpr (Cols) {
          last(gio.template with_out<kOutCond>());  // column passes never scale
        } else {
          if (a.scale) last(gio);  // whole inverse: times L^-1
          else if (a.normalize) last(gio.template with_out<kOutNorm>());
          else last(gio.template with_out<kOutRaw>());
        }
      }
    }
  }
}

template <int Pol, bool Cols, int KH, int KM, int KL, bool TT>
hipError_t launch_k(const KernelArgs &a, int blocks, int threads, size_t lds, hipStream_t stream) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_pass<Pol, Cols, KH, KM, KL, TT>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  hipLaunchKernelGGL((k_pass<Pol, Cols, KH, KM, KL, TT>), dim3(blocks), dim3(threads), lds, stream, a);
  return hipGetLastError();
}

// The split twiddle exists only in the second pass of a transform: the inverse
// column pass and the forward row pass of a split transform.
template <int Pol, bool Cols, int KH, int KM, int KL>
hipError_t launch_tt(bool tt, const KernelArgs &a, int blocks, int threads, size_t lds, hipStream_t stream) {
  if constexpr (Cols != kInverse) {
    (void)tt;
    return launch_k<Pol, Cols, KH, KM, KL, false>(a, blocks, threads, lds, stream);
  } else {
    return tt ? launch_k<Pol, Cols, KH, KM, KL, true>(a, blocks, threads, lds, stream)
              : launch_k<Pol, Cols, KH, KM, KL, false>(a, blocks, threads, lds, stream);
  }
}

// Round splits per word size; must agree with pass_split().
template <int Pol, bool Cols>
hipError_t dispatch_n(int n, bool whole, bool tt, const KernelArgs &a, int blocks, int threads, size_t lds,
                      hipStream_t s) {
#define HNTT_CASE(N, KH, KM, KL) \
  case N: return launch_tt<Pol, Cols, KH, KM, KL>(tt, a, blocks, threads, lds, s);
#if HNTT_WORD == 32
  if constexpr (!Cols) {
    if (whole && (n == 9 || n == 10)) {  // one-pass transforms: a full wave each
      switch (n) {
        HNTT_CASE(9, 3, 3, 3)
        HNTT_CASE(10, 4, 3, 3)
        default: break;
      }
    }
  }
#else
  (void)whole;
#endif
  switch (n) {
    HNTT_CASE(1, 0, 0, 1)
    HNTT_CASE(2, 0, 0, 2)
    HNTT_CASE(3, 0, 0, 3)
    HNTT_CASE(4, 0, 0, 4)
    HNTT_CASE(5, 0, 0, 5)
#if HNTT_WORD == 32
    HNTT_CASE(6, 0, 0, 6)
#else
    HNTT_CASE(6, 3, 0, 3)
#endif
    HNTT_CASE(7, 4, 0, 3)
    HNTT_CASE(8, 4, 0, 4)
#if HNTT_WORD == 32
    HNTT_CASE(9, 5, 0, 4)
    HNTT_CASE(10, 5, 0, 5)
    HNTT_CASE(11, 4, 4, 3)
#else
    HNTT_CASE(9, 3, 3, 3)
    HNTT_CASE(10, 4, 3, 3)
    HNTT_CASE(11, 4, 4, 3)
#endif
    HNTT_CASE(12, 4, 4, 4)
    default: return hipErrorInvalidValue;
  }
#undef HNTT_CASE
}

}  // namespace HNTT_NS

#if HNTT_WORD == 32 && HNTT_INVERSE == 0
#define HNTT_LAUNCH_NAME launch_pass_u32_fwd
#elif HNTT_WORD == 32
#define HNTT_LAUNCH_NAME launch_pass_u32_inv
#elif HNTT_INVERSE == 0
#define HNTT_LAUNCH_NAME launch_pass_u64_fwd
#else
#define HNTT_LAUNCH_NAME launch_pass_u64_inv
#endif

hipError_t HNTT_LAUNCH_NAME(const PassParams &pp, const BatchPtrs &ptrs, hipStream_t stream) {
  const int n = pp.n;
  if (n < 1 || n > kMaxPassLog) return hipErrorInvalidValue;
  const bool cols = pp.kind == PassKind::kCols;
  const int log_other = pp.kind == PassKind::kWhole ? 0 : pp.log_other;
  const int units = (1 << log_other) / pp.group;
  if (units < 1 || pp.nbatch < 1) return hipErrorInvalidValue;
  if (!pp.table && pp.nbatch > kMaxBatchPerLaunch) return hipErrorInvalidValue;
  if (pp.table && (pp.nslots < 1 || pp.nslots > kMaxSlots)) return hipErrorInvalidValue;
  const bool whole = pp.kind == PassKind::kWhole;
  const int threads = pass_tpt(n, HNTT_WORD, whole) * pp.group;
  const size_t lds = pass_lds_bytes(pp);
  if (threads > kMaxPassThreads || (lds == 0 && pass_split(n, HNTT_WORD, whole).kh > 0)) return hipErrorInvalidValue;
  const long long total = (long long)units * pp.nbatch;
  if (total > (1ll << 30)) return hipErrorInvalidValue;
  HNTT_NS::KernelArgs a{};
  a.ptrs = ptrs;
  a.table = pp.table;
  a.units = units;
  a.log_other = log_other;
  a.group = pp.group;
  a.normalize = pp.normalize ? 1 : 0;
  a.scale = (pp.kind == PassKind::kWhole && pp.inverse) ? 1 : 0;
  // the fused product belongs to the final forward pass (rows or whole) only
  if (pp.pm_off && (pp.inverse || pp.kind == PassKind::kCols || !pp.normalize)) return hipErrorInvalidValue;
  if (pp.kind == PassKind::kCols && !pp.inverse && pp.normalize) return hipErrorInvalidValue;
  a.pm_off = pp.pm_off;
  if (pp.zero_upper && (pp.inverse || pp.kind == PassKind::kRows)) return hipErrorInvalidValue;
  a.zero_upper = pp.zero_upper ? 1 : 0;
  if (pp.table) {
    for (int i = 0; i < pp.nslots; ++i) a.slots[i] = pp.slots[i];
  } else {
    a.slots[0] = SlotParams{pp.p, pp.tw, pp.tt, pp.scale_w, pp.scale_wp, pp.jinv, 0};
  }
  const int blocks = (int)total;
  using namespace HNTT_NS;
  const bool tt = pp.table ? pp.slots[0].tt != nullptr : pp.tt != nullptr;
  switch (pp.policy) {
    case kPolicyLazy:
      return cols ? dispatch_n<kPolicyLazy, true>(n, whole, tt, a, blocks, threads, lds, stream)
                  : dispatch_n<kPolicyLazy, false>(n, whole, tt, a, blocks, threads, lds, stream);
    case kPolicyPlain:
      return cols ? dispatch_n<kPolicyPlain, true>(n, whole, tt, a, blocks, threads, lds, stream)
                  : dispatch_n<kPolicyPlain, false>(n, whole, tt, a, blocks, threads, lds, stream);
    case kPolicyMont:
      return cols ? dispatch_n<kPolicyMont, true>(n, whole, tt, a, blocks, threads, lds, stream)
                  : dispatch_n<kPolicyMont, false>(n, whole, tt, a, blocks, threads, lds, stream);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace hntt
