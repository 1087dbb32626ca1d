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
// bits and are read from an LDS copy of the table (from the table in memory, through
// L1, in some forward passes: tw_global); twiddles of the low round
// are uniform across the workgroup (their indices are compile-time multiples of
// 2^(n-1-b)), so they come straight from global memory through scalar loads,
// and the butterflies whose twiddle is 1 skip the product entirely.  The split
// twiddle of a two-pass transform is applied in the row pass in both directions
// (Edge): as words enter the forward row pass, as they leave the inverse one.
// The final forward pass of a polynomial product can multiply its output into a
// partner transform (the pointwise product, GlobalIO::pm) and, in the same
// launch, run the partner's first inverse pass on the product (FUSE).
//
// Row tiles in LDS are laid out against the bank mapping measured on gfx950
// (32-bit accesses: a half-wave per cycle on 32 banks; 16-byte reads: 16 lanes
// per cycle on 64 banks, as four quads of equal lane-bit parity): four pad words
// after every 32, rows of fewer than 32 threads shifted apart (row_skew), and
// the copy-out order of copyout_row_chunk.
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

// Where the rounds read the twiddles that are not compile-time: an LDS copy of the
// per-stage table (Mem = false) or the table in memory through L1/L2 (Mem = true).
template <int Pol, bool Mem>
struct TwSrc {
  static constexpr bool kMem = Mem;
  TwT<Pol> *lds;  // the LDS copy (unused when Mem)
  __device__ __forceinline__ TwT<Pol> at(int i, const HNTT_GLOBAL TwT<Pol> *__restrict__ twg) const {
    if constexpr (Mem) return twg[i];
    else return lds[i];
  }
};

// The modulus of a launch: p, 2p and (Montgomery policy) p^-1 mod beta.
struct Mod {
  T p, p2, j;
};

// Direction of a butterfly, round or edge: forward (Algorithm 1, DIF butterflies)
// or inverse (Algorithm 1 run backwards, DIT butterflies).  Kernels take this
// file's direction (kInverse); a kernel that runs both takes each explicitly.
template <int Pol, bool INV = kInverse>
__device__ __forceinline__ void bfly(T &x, T &y, const TwT<Pol> &tw, const Mod &m) {
  if constexpr (Pol == kPolicyMont) {
    if constexpr (INV) bfly_inv_mont<Wd>(x, y, tw, m.p, m.p2, m.j);
    else bfly_fwd_mont<Wd>(x, y, tw, m.p, m.p2, m.j);
  } else if constexpr (INV) {
    if constexpr (Pol == kPolicyLazy) bfly_inv_lazy<Wd>(x, y, tw.x, tw.y, m.p, m.p2);
    else bfly_inv_plain<Wd>(x, y, tw.x, tw.y, m.p);
  } else {
    if constexpr (Pol == kPolicyLazy) bfly_fwd_lazy<Wd>(x, y, tw.x, tw.y, m.p, m.p2);
    else bfly_fwd_plain<Wd>(x, y, tw.x, tw.y, m.p);
  }
}

// Butterfly whose twiddle is 1: no product (both lazy policies share the ranges).
template <int Pol, bool INV = kInverse>
__device__ __forceinline__ void bfly_w1(T &x, T &y, const Mod &m) {
  if constexpr (INV) {
    if constexpr (Pol != kPolicyPlain) bfly_inv_lazy_w1<Wd>(x, y, m.p2);
    else bfly_inv_plain_w1<Wd>(x, y, m.p);
  } else {
    if constexpr (Pol != kPolicyPlain) bfly_fwd_lazy_w1<Wd>(x, y, m.p2);
    else bfly_fwd_plain_w1<Wd>(x, y, m.p);
  }
}

// x (any word) times a table constant, result in [0,2p).
template <int Pol, bool INV = kInverse>
__device__ __forceinline__ T mul_const(T x, const TwT<Pol> &tw, const Mod &m) {
  if constexpr (Pol == kPolicyMont) return mont_lazy<Wd>(x, tw, m.p, m.j);
  else if constexpr (!INV) return shoup_lazy<Wd>(x, tw.x, tw.y, m.p);
  else return shoup_lazy_sub<Wd>(x, tw.x, tw.y, m.p);
}

// Forward row passes: fold the split twiddle's low factor into the high round, and
// read its high factors from the LDS row pads.
constexpr bool kFwdFold = false;
constexpr bool kFwdHiLds = true;

// Words per 16-byte vector access.
constexpr int kVec = 16 / sizeof(T);

// One round of K stages on the position bits [b_lo, b_lo + K).  Stage i of
// Algorithm 1 pairs bit b = n - i; its twiddle is zeta_i^(pos mod 2^b), which is
// entry (1 << b) + (pos mod 2^b) of the per-stage ("heap") table, so that lanes
// with consecutive positions read consecutive entries.
// LowRound: b_lo = 0, the twiddle indices are compile-time constants and are
// read from global memory with scalar loads; the butterflies with twiddle 1
// skip the product.  Otherwise the twiddles come from `tws` (the LDS copy of the
// table, or the table in memory: TwSrc).
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

// Fold of a per-thread factor A into one stage of the row pass's high round.  A
// round's stages are linear in the thread's words, so a factor common to all of
// them (the split twiddle's low factor, which depends only on the row and on the
// thread's low position bits) may be applied at either end of the round and
// merged into the stage there, whose butterflies all have the same twiddle W
// (its index is the thread's low position bits):
//   forward (DIF), the round's last stage: (X, Y) -> (X + Y, W (X - Y)) becomes
//   (A (X + Y), (A W) (X - Y)), with no conditional subtraction before the
//   product by A (a product accepts any input below beta);
//   inverse (DIT), the round's first stage: (X, Y) -> (X + W Y, X - W Y) becomes
//   (A X + (A W) Y, A X - (A W) Y), where the product A X also takes the place
//   of Algorithm 4's conditional subtraction of X.
// Either way one product by A and one by the precomputed A W replace the product
// by W and two products by A.
struct NoFold {
  static constexpr bool kOn = false;
};
template <int Pol>
struct Fold {
  static constexpr bool kOn = true;
  TwT<Pol> a, aw;
};

template <int Pol>
__device__ __forceinline__ void bfly_fold(T &x, T &y, const TwT<Pol> &a, const TwT<Pol> &aw, const Mod &m) {
  if constexpr (Pol == kPolicyPlain) {  // X, Y in [0,p): every output fully reduced
    T d = x - y;
    const T dp = d + m.p;
    d = dp < d ? dp : d;
    x = csub<T>(mul_const<Pol, false>(x + y, a, m), m.p);
    y = csub<T>(mul_const<Pol, false>(d, aw, m), m.p);
  } else {  // X, Y in [0,2p): X + Y < 4p and X - Y + 2p < 4p are below beta
    const T t = x - y + m.p2;
    x = mul_const<Pol, false>(x + y, a, m);
    y = mul_const<Pol, false>(t, aw, m);
  }
}

template <int Pol>
__device__ __forceinline__ void bfly_fold_inv(T &x, T &y, const TwT<Pol> &a, const TwT<Pol> &aw, const Mod &m) {
  if constexpr (Pol == kPolicyPlain) {  // X, Y in [0,p): every output fully reduced
    const T xr = csub<T>(mul_const<Pol, true>(x, a, m), m.p);
    const T t = csub<T>(mul_const<Pol, true>(y, aw, m), m.p);
    T d = xr - t;
    const T dp = d + m.p;
    y = dp < d ? dp : d;
    x = csub<T>(xr + t, m.p);
  } else {  // X, Y in [0,4p) (Theorem 3 ranges); both products in [0,2p)
    const T xr = mul_const<Pol, true>(x, a, m);
    const T t = mul_const<Pol, true>(y, aw, m);
    x = xr + t;
    y = xr - t + m.p2;
  }
}

// A source whose words are loaded raw and finished (the split twiddle applied)
// only after the round's hook, so that the loads can be issued before a barrier
// that the finishing step needs (its factors staged in LDS).
template <class S, class = void>
struct DefersIn {
  static constexpr bool value = false;
};
template <class S>
struct DefersIn<S, std::void_t<decltype(S::kDeferIn)>> {
  static constexpr bool value = S::kDeferIn;
};

// The K stages of one round on a thread's 2^K words v (positions base | (e << b_lo)).
template <int Pol, int N_LOG, int K, bool LowRound, bool INV, class FoldT, class TwS>
__device__ __forceinline__ void round_stages(T (&v)[1 << K], int b_lo, int base, const TwS &tws,
                                            const HNTT_GLOBAL TwT<Pol> *__restrict__ twg, const Mod &m,
                                            const FoldT &fold) {
  constexpr int M = 1 << K;
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const int hb = INV ? s : K - 1 - s;
#pragma unroll
      for (int e = 0; e < M; ++e) {
        if (e & (1 << hb)) continue;
        if constexpr (FoldT::kOn) {
          if (s == (INV ? 0 : K - 1)) {  // the stage pairing bit b_lo (hb = 0), the thread's factor folded in
            if constexpr (INV) bfly_fold_inv<Pol>(v[e], v[e | 1], fold.a, fold.aw, m);
            else bfly_fold<Pol>(v[e], v[e | 1], fold.a, fold.aw, m);
            continue;
          }
        }
        if constexpr (LowRound) {
          const int kk = e & ((1 << hb) - 1);
          if (kk == 0) {
            bfly_w1<Pol, INV>(v[e], v[e | (1 << hb)], m);
          } else {
            const TwT<Pol> tw = twg[(1 << hb) + kk];
            bfly<Pol, INV>(v[e], v[e | (1 << hb)], tw, m);
          }
        } else {
          const int b = b_lo + hb;
          const int pos = base | (e << b_lo);
          const int ti = (1 << b) + (pos & ((1 << b) - 1));
          const TwT<Pol> tw = tws.at(ti, twg);
          bfly<Pol, INV>(v[e], v[e | (1 << hb)], tw, m);
        }
      }
    }
}

// Optional work on a round's words after its stages and before they are stored
// (the fused pointwise product and inverse stages of a polynomial product).
struct NoMid {
  static constexpr bool kOn = false;
};

template <int Pol, int N_LOG, int K, bool LowRound, bool ZU = false, class Src, class Dst, class Hook = NoHook,
          class FoldT = NoFold, bool INV = kInverse, class MidT = NoMid, class TwS>
__device__ __forceinline__ void round_k(int b_lo, int t, int tpt, const TwS &tws,
                                       const HNTT_GLOBAL TwT<Pol> *__restrict__ twg, const Mod &m, const Src &src,
                                       const Dst &dst, const Hook &after_load = Hook{}, const FoldT &fold = FoldT{},
                                       const MidT &mid = MidT{}) {
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
    } else if constexpr (DefersIn<Src>::value) {
#pragma unroll
      for (int e = 0; e < M; ++e) v[e] = (ZU && ((e >> (K - 1)) & 1)) ? (T)0 : src.load_raw(base, e << b_lo);
    } else {
#pragma unroll
      for (int e = 0; e < M; ++e) v[e] = (ZU && ((e >> (K - 1)) & 1)) ? (T)0 : src.load2(base, e << b_lo);
    }
    // Every thread runs groups / tpt >= 1 iterations, so a hook that synchronises
    // the workgroup is reached once by all threads.
    if (gi == t) {
      after_load();
      if constexpr (INV) __builtin_amdgcn_s_setprio(0);  // raised at the start of an inverse k_pass
    }
    if constexpr (DefersIn<Src>::value) {
#pragma unroll
      for (int e = 0; e < M; ++e)
        if (!(ZU && ((e >> (K - 1)) & 1))) v[e] = src.finish(v[e], base, e << b_lo);
    }
    round_stages<Pol, N_LOG, K, LowRound, INV>(v, b_lo, base, tws, twg, m, fold);
    if constexpr (MidT::kOn) mid(v, base);
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
template <int Pol, bool INV = kInverse>
__device__ __forceinline__ T reduce_final(T x, T p) {
  if constexpr (Pol == kPolicyPlain) return x;
  if constexpr (INV) x = csub<T>(x, p + p);
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

// The fused pointwise product of a final forward pass: x times the partner's word
// ab = A beta mod p in [0,p) (the partner operand was prepared times beta, so its
// transform carries the factor beta), for any x < beta: one Montgomery product
// x ab beta^-1 = x A mod p, in (0,2p), which the lazy inverse accepts as it is;
// the plain policy reduces it to [0,p).
template <int Pol>
__device__ __forceinline__ T pmul_word(T x, T ab, const Mod &m) {
  const T u = mont_lazy<Wd>(x, ab, m.p, m.j);
  return Pol == kPolicyPlain ? csub<T>(u, m.p) : u;
}

// Split-twiddle factors held in the pad words of an LDS row tile (four pad words
// after every 32 words of a row, never touched by the tile exchange): factor e of
// a row sits in pad block e / kPadTw, kPadTw factors per block.
constexpr int kTwRatio(int pol) { return pol == kPolicyMont ? 1 : 2; }  // words per table entry
template <int Pol>
__device__ __forceinline__ int pad_slot(int e) {
  constexpr int r = kTwRatio(Pol), per = 4 / r;
  return (e / per) * (36 / r) + 32 / r + e % per;
}

// The middle of a fused polynomial-product row (or whole) pass, run on the words
// of the forward transform's low round while they are still in registers: the
// pointwise product with the partner transform A's words at the same positions
// (read from memory, fully reduced), then the inverse transform's low-round
// stages (DIT, compile-time twiddles of the inverse table), so that the words can
// go back to the same thread-private places of the LDS tile.
template <int Pol, int N_LOG, int K>
struct FusedMid {
  static constexpr bool kOn = true;
  const HNTT_GLOBAL T *a_sub;                     // A's words of this sub-transform
  const HNTT_GLOBAL TwT<Pol> *__restrict__ twg_i;  // inverse per-stage table
  Mod m;
  __device__ __forceinline__ void operator()(T (&v)[1 << K], int base) const {
    constexpr int M = 1 << K;
    if constexpr (M >= kVec) {
      Vec16 q[M / kVec];
#pragma unroll
      for (int e = 0; e < M; e += kVec) q[e / kVec] = *reinterpret_cast<const HNTT_GLOBAL Vec16 *>(a_sub + base + e);
#pragma unroll
      for (int e = 0; e < M; e += kVec) {
        const T *w = reinterpret_cast<const T *>(&q[e / kVec]);
#pragma unroll
        for (int i = 0; i < kVec; ++i) v[e + i] = pmul_word<Pol>(v[e + i], w[i], m);
      }
    } else {
#pragma unroll
      for (int e = 0; e < M; ++e) v[e] = pmul_word<Pol>(v[e], a_sub[base + e], m);
    }
    round_stages<Pol, N_LOG, K, true, true>(v, 0, base, nullptr, twg_i, m, NoFold{});
  }
};

// What happens to a word on its way in from HBM and out to HBM.  The split
// twiddle of a two-pass transform (the factor omega^(s pos) between the column
// and the row transforms of an R x C view, s the bit-reversed row index) is
// applied in the row pass, for both directions: forward, to row s's
// word at position pos as it is loaded (before the row transform); inverse, as
// it is stored (after the row transform, with the conjugate root and L^-1).  It
// is the product of two factors, one indexed by the low SIGMA bits of the
// position and one by the remaining high bits, from a per-row table
// [low factors (2^SIGMA) | high factors (2^(n-SIGMA)) | folded low factors (2^SIGMA)].
// SIGMA is the bit boundary of the row pass's high register round, so the low
// factor is fixed per thread in that round and the high factor is shared by all
// lanes of a row.  TT = false: no split twiddle.
// LO = false: the low factor is not applied here but folded into the high round's
// stage next to the split twiddle (see Fold).  HI_LDS: the high factors of the
// thread's row come from the pads of its LDS tile (hi_lds), staged with the
// per-stage twiddle table, instead of from the table in memory.
// Out fixes what out() does: kOutRaw passes words through (the first pass of a
// two-pass transform), kOutNorm reduces them to [0,p), kOutCond reduces them
// with p replaced by 0 when normalisation is off (the same instructions either
// way, no select), kOutAny follows the runtime flags (whole inverse transforms,
// which may also scale by L^-1).  The final round of a pass picks its variant
// with one uniform branch: with the flags tested per word, the compiler computes
// the reduction for every word and selects afterwards, also when it is not wanted.
constexpr int kOutRaw = 0, kOutNorm = 1, kOutAny = 2, kOutCond = 3;
template <int Pol, bool Cols, bool TT, int N_LOG, int SIGMA, int Out = kOutAny, bool LO = true, bool HI_LDS = false,
          bool INV = kInverse>
struct Edge {
  static constexpr bool kInv = INV;
  static constexpr int kPol = Pol;
  Mod m;
  int normalize, scale;
  T sw, swp;
  __amdgpu_buffer_rsrc_t tt;  // factor tables of the pass
  uint32_t tt_off;            // byte offset of this row's first factor
  const TwT<Pol> *hi_lds;     // HI_LDS: this row's tile base in LDS (table-entry units)
  // the split twiddle of position pos = lp + up (disjoint bits: lp varies per lane,
  // up is uniform), times x; any x below beta, result in [0,2p) ([0,p): plain)
  __device__ __forceinline__ T twist(T x, int lp, int up) const {
    constexpr uint32_t kTw = sizeof(TwT<Pol>);
    constexpr int kMask = (1 << SIGMA) - 1;
    TwT<Pol> hi;
    if constexpr (HI_LDS) hi = hi_lds[pad_slot<Pol>((lp >> SIGMA) + (up >> SIGMA))];
    else hi = buf_load_tw<Pol>(tt, tt_off + (uint32_t)((1 << SIGMA) + (lp >> SIGMA)) * kTw, (uint32_t)(up >> SIGMA) * kTw);
    x = mul_const<Pol, INV>(x, hi, m);
    if constexpr (LO) {
      const TwT<Pol> lo = buf_load_tw<Pol>(tt, tt_off + (uint32_t)(lp & kMask) * kTw, (uint32_t)(up & kMask) * kTw);
      x = mul_const<Pol, INV>(x, lo, m);
    }
    if constexpr (Pol == kPolicyPlain) x = csub<T>(x, m.p);
    return x;
  }
  __device__ __forceinline__ T in(T x, int lp, int up) const {
    if constexpr (TT && !INV) x = twist(x, lp, up);
    return x;
  }
  __device__ __forceinline__ T in(T x, int pos) const { return in(x, pos, 0); }
  template <int O>
  __device__ __forceinline__ Edge<Pol, Cols, TT, N_LOG, SIGMA, O, LO, HI_LDS, INV> with_out() const {
    return {m, normalize, scale, sw, swp, tt, tt_off, hi_lds};
  }
  // pos = lp + up as in twist(); the split twiddle of an inverse row pass, then the
  // output reduction
  __device__ __forceinline__ T out(T x, int lp, int up) const {
    if constexpr (TT && INV) x = twist(x, lp, up);
    return reduce_out(x);
  }
  __device__ __forceinline__ T out(T x, int pos) const { return out(x, pos, 0); }
  __device__ __forceinline__ T reduce_out(T x) const {
    if constexpr (Out == kOutRaw) {
      return x;
    } else if constexpr (Out == kOutNorm) {
      return reduce_final<Pol, INV>(x, m.p);
    } else if constexpr (Out == kOutCond) {
      return reduce_final<Pol, INV>(x, normalize ? m.p : (T)0);
    } else if constexpr (!Cols && INV) {
      if (scale) {  // whole inverse transform: times L^-1, then reduced
        if constexpr (Pol == kPolicyMont) x = mont_lazy<Wd>(x, sw, m.p, m.j);
        else x = shoup_lazy_sub<Wd>(x, sw, swp, m.p);
        if (normalize) x = csub<T>(x, m.p);
      } else if (normalize) {
        x = reduce_final<Pol, INV>(x, m.p);
      }
    } else {
      if (normalize) x = reduce_final<Pol, INV>(x, m.p);
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
    g.rsrc = rsrc;
    g.off = off;
    g.stride = stride;
    g.edge = edge.template with_out<O>();
    return g;
  }
  __device__ __forceinline__ T load_raw(int lp, int up) const {
    if constexpr (Cols) {
      return buf_load(rsrc, (off + (uint32_t)lp * stride) * (uint32_t)sizeof(T),
                      (uint32_t)up * stride * (uint32_t)sizeof(T));
    } else {
      return base[off + (uint32_t)(lp + up)];
    }
  }
  __device__ __forceinline__ T load2(int lp, int up) const { return edge.in(load_raw(lp, up), lp, up); }
  __device__ __forceinline__ void store2(int lp, int up, T x) const {
    x = edge.out(x, lp, up);
    if constexpr (!Cols && !EdgeT::kInv) {  // (the fused product ends forward transforms only)
      if (pm) {
        HNTT_GLOBAL T *q = pm + off + (uint32_t)(lp + up);
        *q = pmul_word<EdgeT::kPol>(x, *q, edge.m);
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
    if (!EdgeT::kInv && pm) {
      HNTT_GLOBAL Vec16 *dst = reinterpret_cast<HNTT_GLOBAL Vec16 *>(pm + (off + (uint32_t)pos));
      const Vec16 pa = *dst;
      const T *pw = reinterpret_cast<const T *>(&pa);
#pragma unroll
      for (int i = 0; i < kVec; ++i) w[i] = pmul_word<EdgeT::kPol>(w[i], pw[i], edge.m);
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

// A global source read raw, its input edge applied after the round's hook (DefersIn).
template <class IO>
struct DeferredIn {
  static constexpr bool kContig = IO::kContig;
  static constexpr bool kDeferIn = true;
  IO io;
  __device__ __forceinline__ T load_raw(int lp, int up) const { return io.load_raw(lp, up); }
  __device__ __forceinline__ T finish(T x, int lp, int up) const { return io.edge.in(x, lp, up); }
};

// Copy of the N-entry heap twiddle table into LDS, in two steps so that its global
// loads are in flight together with the tile's: load() issues up to kR loads per
// thread into registers, store() writes them to LDS (and copies any remainder).
template <int Pol, int N, bool Mem>
struct TwStage {
  static constexpr int N_LOG2 = __builtin_ctz(N);
  static constexpr int kR = 8;
  TwT<Pol> r[kR];
  int nthr;  // threads in the workgroup
  __device__ __forceinline__ void load(const HNTT_GLOBAL TwT<Pol> *__restrict__ twg) {
    if constexpr (Mem) return;
#pragma unroll
    for (int j = 0; j < kR; ++j) {
      const int i = threadIdx.x + j * nthr;
      if (i < N) r[j] = twg[i];
    }
  }
  __device__ __forceinline__ void store(TwT<Pol> *tws, const HNTT_GLOBAL TwT<Pol> *__restrict__ twg) const {
    if constexpr (Mem) return;
#pragma unroll
    for (int j = 0; j < kR; ++j) {
      const int i = threadIdx.x + j * nthr;
      if (i < N) tws[i] = r[j];
    }
    for (int i = threadIdx.x + kR * nthr; i < N; i += nthr) tws[i] = twg[i];
  }
};

// The 16-byte chunk of a row that copy-in or copy-out slot q moves.  A row tile in LDS has
// four pad words after every 32 words, so 16 consecutive chunks span 17 or 18
// 16-byte units and two of them meet in one bank when a 16-lane group of a
// 16-byte read covers 256 bytes of banks.  Slots are therefore dealt in groups
// of 16 whose first eight take one 32-word block (8 chunks) and whose last eight
// the block eight blocks later (8 x 36 words on, i.e. half the banks across):
// each 16-lane group reads 64 distinct banks, and each eight lanes still store
// 128 contiguous bytes.  32-bit words only: with 64-bit words 16 consecutive
// chunks already fall in distinct banks.
template <int kChunks>
__device__ __forceinline__ int copyout_chunk(int q) {
  if constexpr (kVec == 4 && kChunks >= 128) {
    const int l = q & 15, pr = q >> 4;
    const int blk = (pr & 7) + ((pr >> 3) << 4) + ((l >> 3) << 3);
    return (blk << 3) | (l & 7);
  } else {
    return q;
  }
}

// The chunk that thread t of row g moves in step j of a row pass's copy-out (the
// tile read from LDS with 16-byte loads, written out with eight lanes on each 128
// contiguous bytes).  A 16-byte LDS read serves 16 lanes per cycle on 64 banks:
// four quads of four lanes, the quads of one half-wave whose lane bits 2-4 have the
// same parity.  With 32 threads per row (2^10 words), the four 8-lane segments of
// step j take 32-word blocks j, j + 16, j + 8 and j + 24, whose bank offsets (36
// words per block) are x, x, x + 32, x + 32: each quad group then covers the 64
// banks once.  With 16 threads per row (2^9 words: two rows per half-wave, rows
// TPT words apart) the segments take blocks j and j + 8, turned by 12 blocks in
// odd rows, and with 2^8 words blocks j and j + 4, turned by 4.  Other shapes keep
// copyout_chunk's order.
template <int kChunks, int TPT>
__device__ __forceinline__ int copyout_row_chunk(int t, int j, int g) {
  if constexpr (kVec == 4 && TPT == 32 && kChunks == 256) {
    const int k = t >> 3;
    const int perm = ((k & 1) << 1) | (k >> 1);  // 0, 2, 1, 3
    return ((j + 8 * perm) << 3) | (t & 7);
  } else if constexpr (kVec == 4 && TPT == 16 && (kChunks == 128 || kChunks == 64)) {
    constexpr int kBlk = kChunks / 8, kPerSeg = kBlk / 2, kTurn = kChunks == 128 ? 12 : 4;
    const int blk = (j + kPerSeg * (t >> 3) + kTurn * (g & 1)) & (kBlk - 1);
    return (blk << 3) | (t & 7);
  } else {
    return copyout_chunk<kChunks>(t + j * TPT);
  }
}

// An exchange through LDS among the lanes of one wave: the wave's LDS operations
// complete in order, so only the compiler must be kept from moving them across.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Padded LDS words per sub-transform (rows: row pitch; cols: rows of the tile).
template <bool Cols>
constexpr int padded_len(int N) {
  return Cols ? N + N / 32 : (int)row_padded_len((size_t)N);
}

// Waves per SIMD that a pass's LDS tile allows, given to the compiler so that it
// schedules for that occupancy instead of squeezing registers for more waves
// than the LDS can host (a 2^5-word-per-thread tile of 32-bit words, or 2^4 of
// 64-bit words, takes about 144 bytes of LDS per thread: four waves per SIMD).
// Other passes (no tile, or a tile that leaves room for more waves than their
// registers do): the default range.
constexpr bool pass_big_tile(int kh, int km, int kl) {
  const int kmax = kh > kl ? (kh > km ? kh : km) : (kl > km ? kl : km);
  return kh > 0 && (1 << kmax) * (int)sizeof(T) >= 128;
}
constexpr int pass_waves_min(int kh, int km, int kl) { return pass_big_tile(kh, km, kl) ? 4 : 1; }
constexpr int pass_waves_max(int kh, int km, int kl) { return pass_big_tile(kh, km, kl) ? 4 : 8; }

// FUSE (32-bit forward row or whole passes of a polynomial product): after the
// forward transform of B_k's sub-transform, multiply by A_k's words (A_k starts
// pm_off words earlier), run the inverse transform of the same sub-transform on
// the product and write it over A_k (see FusedMid).
template <int Pol, bool Cols, int KH, int KM, int KL, bool TT, bool FUSE = false>
__global__ void __launch_bounds__(kMaxPassThreads)
    __attribute__((amdgpu_waves_per_eu(pass_waves_min(KH, KM, KL), pass_waves_max(KH, KM, KL))))
    k_pass(KernelArgs a) {
  constexpr int N_LOG = KH + KM + KL;
  // bit boundary of the high register round (split-twiddle factorisation of a row pass)
  constexpr int SIGMA = KM + KL;
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
  // the high and middle rounds' twiddles: from memory in some forward passes (a row
  // pass carries the split twiddle, a whole-transform pass does not), else from an
  // LDS copy of the table placed before the tile
  constexpr bool kTwMem = tw_global(N_LOG, HNTT_WORD, !Cols && !kInverse, !Cols && !TT);
  TwT<Pol> *const tw_lds = reinterpret_cast<TwT<Pol> *>(smem_raw);
  const TwSrc<Pol, kTwMem> tws{tw_lds};
  T *tile = kTwMem ? reinterpret_cast<T *>(smem_raw) : reinterpret_cast<T *>(tw_lds + N);

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
    // Row passes with a high register round fold the split twiddle's low factor into
    // that round (Fold) and, where the row tile's pads hold them, read the high
    // factors from LDS.
    constexpr bool kFold = TT && !Cols && KH > 0 && (kInverse || kFwdFold);
    // rows whose threads all belong to one wave (consecutive thread ids)
    constexpr bool kRowInWave = !Cols && TPT <= 64;
    // The rows of one wave read the same factor index at once; their pads would sit
    // in the same bank (the row pitch is a multiple of 64 words), so row g's factors
    // start (g mod rows-per-wave) pad blocks later: 36 words, i.e. another bank.
    constexpr int kRowsPerWave = TPT >= 64 ? 1 : 64 / TPT;
    constexpr int kPadTw = 4 / kTwRatio(Pol);  // factors per pad block
    constexpr bool kHiLds = TT && !Cols && KH > 0 && (kInverse || kFwdHiLds) &&
                            (1 << KH) + (kRowsPerWave - 1) * kPadTw <= (N / 32) * kPadTw;
    using EdgeT = Edge<Pol, Cols, TT, N_LOG, SIGMA, kOutAny, !kFold, kHiLds>;
    // LDS pitch of a row tile (columns: of a column segment)
    constexpr int kPitchT = padded_len<Cols>(N) + (Cols ? 0 : (int)row_skew(N_LOG, KH, KM, KL, 8 * sizeof(T)));
    EdgeT edge{m, a.normalize, a.scale, (T)sp.scale_w, (T)sp.scale_wp, make_rsrc(sp.tt, 0), 0, nullptr};
    GlobalIO<Cols, EdgeT> gio;
    constexpr uint32_t kTw = sizeof(TwT<Pol>);
    // factors per row: low, high, folded low
    constexpr uint32_t kTTStride = 2u * (1u << SIGMA) + (1u << (N_LOG - SIGMA));
    if constexpr (TT)
      edge.tt = make_rsrc((const void *)uniform64((uint64_t)sp.tt), (1u << a.log_other) * kTTStride * kTw);
    gio.base = gbase;
    gio.pm = a.pm_off ? gbase - a.pm_off : nullptr;
    if constexpr (Cols) {
      const uint32_t col = (uint32_t)unit * G + g;
      gio.rsrc = make_rsrc((const void *)gbase, (uint32_t)(C * N * sizeof(T)));
      gio.off = col;
      gio.stride = (uint32_t)C;
    } else {
      const uint32_t row = (uint32_t)unit * G + g;
      gio.off = row * N;
      gio.stride = 1;
      edge.tt_off = row * kTTStride * kTw;
      if constexpr (kHiLds)
        edge.hi_lds = reinterpret_cast<const TwT<Pol> *>(tile + g * kPitchT) + (g % kRowsPerWave) * (36 / kTwRatio(Pol));
    }
    gio.edge = edge;
    // the thread's low factor A and A W for the stage that pairs bit SIGMA (its
    // twiddle W is the same for all of the thread's butterflies in that stage)
    using FoldT = std::conditional_t<kFold, Fold<Pol>, NoFold>;
    FoldT fold{};
    if constexpr (kFold) {
      const uint32_t lo = (uint32_t)t & ((1u << SIGMA) - 1);
      fold.a = buf_load_tw<Pol>(edge.tt, edge.tt_off + lo * kTw, 0);
      fold.aw = buf_load_tw<Pol>(edge.tt, edge.tt_off + ((1u << SIGMA) + (1u << (N_LOG - SIGMA)) + lo) * kTw, 0);
    }
    // High factors of the workgroup's G rows into the pads of their LDS rows: loaded
    // with the per-stage twiddle table, written with it before the same barrier.
    constexpr int kHiPer = kHiLds ? ((KH + KMAX - N_LOG) > 0 ? 1 << (KH + KMAX - N_LOG) : 1) : 1;
    TwT<Pol> hreg[kHiPer];
    const auto hi_load_from = [&](__amdgpu_buffer_rsrc_t tbl) {
      if constexpr (kHiLds) {
        const int nthr = G * TPT;
#pragma unroll
        for (int j = 0; j < kHiPer; ++j) {
          const int i = threadIdx.x + j * nthr;
          if (i < (G << KH)) {
            const uint32_t row = (uint32_t)unit * G + (uint32_t)(i >> KH);
            hreg[j] = buf_load_tw<Pol>(tbl, (row * kTTStride + (1u << SIGMA) + (uint32_t)(i & ((1 << KH) - 1))) * kTw, 0);
          }
        }
      }
    };
    const auto hi_load = [&]() { hi_load_from(edge.tt); };
    // Fused polynomial product (FUSE): the inverse side of the same sub-transform,
    // written over the partner A_k.  Its split twiddle (rows) is folded and its high
    // factors come from the row pads exactly as the forward ones.
    constexpr bool kFoldI = FUSE && TT && KH > 0;
    constexpr bool kHiLdsI = FUSE && kHiLds;
    static_assert(kFoldI || !kHiLdsI, "LDS high factors go with the fold");
    using EdgeI = Edge<Pol, false, TT, N_LOG, SIGMA, kOutAny, !kFoldI, kHiLdsI, true>;
    const HNTT_GLOBAL TwT<Pol> *__restrict__ twg_i = (const HNTT_GLOBAL TwT<Pol> *)(sp.tw2);
    EdgeI edge_i{m, a.normalize, a.scale, (T)sp.scale_w, (T)sp.scale_wp, make_rsrc(sp.tt2, 0), 0, nullptr};
    GlobalIO<false, EdgeI> gio_a;
    using FoldI = std::conditional_t<kFoldI, Fold<Pol>, NoFold>;
    FoldI fold_i{};
    FusedMid<Pol, N_LOG, KL> fmid{};
    if constexpr (FUSE) {
      static_assert(!Cols && !kInverse && sizeof(T) == 4 && Pol != kPolicyMont,
                    "the fused product runs on 32-bit forward row or whole passes (Shoup policies)");
      const uint32_t row = (uint32_t)unit * G + g;
      if constexpr (TT)
        edge_i.tt = make_rsrc((const void *)uniform64((uint64_t)sp.tt2), (1u << a.log_other) * kTTStride * kTw);
      edge_i.tt_off = row * kTTStride * kTw;
      if constexpr (kHiLdsI)
        edge_i.hi_lds = reinterpret_cast<const TwT<Pol> *>(tile + g * kPitchT) + (g % kRowsPerWave) * (36 / kTwRatio(Pol));
      HNTT_GLOBAL T *const abase = gbase - a.pm_off;
      gio_a.base = abase;
      gio_a.pm = nullptr;
      gio_a.off = row * N;
      gio_a.stride = 1;
      gio_a.edge = edge_i;
      fmid = FusedMid<Pol, N_LOG, KL>{abase + (size_t)row * N, twg_i, m};
    }
    const auto hi_store = [&]() {
      if constexpr (kHiLds) {
        const int nthr = G * TPT;
        TwT<Pol> *const tile_tw = reinterpret_cast<TwT<Pol> *>(tile);
#pragma unroll
        for (int j = 0; j < kHiPer; ++j) {
          const int i = threadIdx.x + j * nthr;
          if (i < (G << KH)) {
            const int gg = i >> KH;
            tile_tw[gg * (kPitchT / kTwRatio(Pol)) + (gg % kRowsPerWave) * (36 / kTwRatio(Pol)) +
                    pad_slot<Pol>(i & ((1 << KH) - 1))] = hreg[j];
          }
        }
      }
    };

    if constexpr (KH == 0 && FUSE) {
      // one round: B_k's words, forward stages, times A_k's words, inverse stages, into A_k
      if (a.zero_upper)
        round_k<Pol, N_LOG, KL, true, true, decltype(gio), decltype(gio_a), NoHook, NoFold, false>(
            0, t, TPT, nullptr, twg, m, gio, gio_a, NoHook{}, NoFold{}, fmid);
      else
        round_k<Pol, N_LOG, KL, true, false, decltype(gio), decltype(gio_a), NoHook, NoFold, false>(
            0, t, TPT, nullptr, twg, m, gio, gio_a, NoHook{}, NoFold{}, fmid);
    } else if constexpr (KH == 0) {
      // one round, HBM to HBM
      if (!kInverse && a.zero_upper) round_k<Pol, N_LOG, KL, true, true>(0, t, TPT, nullptr, twg, m, gio, gio);
      else round_k<Pol, N_LOG, KL, true>(0, t, TPT, nullptr, twg, m, gio, gio);
    } else {
      // The twiddle table's loads are issued first and written to LDS only after
      // the tile's loads are in flight: one memory round trip before the stages.
      const int nthr = G * TPT;  // blockDim.x
      TwStage<Pol, N, kTwMem> stage;
      stage.nthr = nthr;
      stage.load(twg);
      hi_load();
      const LdsIO<Cols> lio{tile, G, g, kPitchT};
      if constexpr (!kInverse) {
        // Rows with fewer than 32 threads per row: a high-round load instruction would
        // cover under 128 bytes of each row, so the tile is first copied into LDS with
        // consecutive lanes on consecutive 16 bytes, and the high round reads it there.
        constexpr bool kCopyIn = !Cols && TPT < 32;
        if constexpr (kCopyIn) {
          constexpr int kPitch = kPitchT;
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
            // each thread moves chunks t + j TPT of its own row g
            Vec16 q[kLoad];
#pragma unroll
            for (int j = 0; j < kLoad; ++j)
              q[j] = *reinterpret_cast<const HNTT_GLOBAL Vec16 *>(rows0 + (size_t)g * N +
                                                                   copyout_chunk<kCh>(t + j * TPT) * kVec);
#pragma unroll
            for (int j = 0; j < kLoad; ++j) {
              const int c = copyout_chunk<kCh>(t + j * TPT) * kVec;
              *reinterpret_cast<Vec16 *>(tile + g * kPitch + c + ((c >> 5) << 2)) = q[j];
            }
            stage.store(tw_lds, twg);
            hi_store();
            __syncthreads();  // tile, twiddle table and high factors staged
            const LdsEdgeIO<EdgeT> lin{lio, edge};
            round_k<Pol, N_LOG, KH, false, ZU>(KM + KL, t, TPT, tws, twg, m, lin, lio, NoHook{}, fold);
          };
          if (a.zero_upper) copy_in(std::true_type{});
          else copy_in(std::false_type{});
        } else if constexpr (TT && kHiLds) {
          // the row's words are loaded raw, the twiddle table and high factors are
          // staged meanwhile, and the split twiddle is applied after the barrier
          const auto staged = [&]() {
            stage.store(tw_lds, twg);
            hi_store();
            __syncthreads();  // twiddle table and high factors staged
          };
          const DeferredIn<decltype(gio)> din{gio};
          if (a.zero_upper) round_k<Pol, N_LOG, KH, false, true>(KM + KL, t, TPT, tws, twg, m, din, lio, staged, fold);
          else round_k<Pol, N_LOG, KH, false>(KM + KL, t, TPT, tws, twg, m, din, lio, staged, fold);
        } else if constexpr (TT) {
          // the split twiddle's products follow the loads and would all have to
          // finish before a barrier placed after them: the table goes first
          stage.store(tw_lds, twg);
          hi_store();
          __syncthreads();  // twiddle table and high factors staged
          if (a.zero_upper) round_k<Pol, N_LOG, KH, false, true>(KM + KL, t, TPT, tws, twg, m, gio, lio, NoHook{}, fold);
          else round_k<Pol, N_LOG, KH, false>(KM + KL, t, TPT, tws, twg, m, gio, lio, NoHook{}, fold);
        } else {
          const auto staged = [&]() {
            stage.store(tw_lds, twg);
            __syncthreads();  // twiddle table staged
          };
          if (a.zero_upper) round_k<Pol, N_LOG, KH, false, true>(KM + KL, t, TPT, tws, twg, m, gio, lio, staged);
          else round_k<Pol, N_LOG, KH, false>(KM + KL, t, TPT, tws, twg, m, gio, lio, staged);
        }
        // A row no wider than a wave exchanges among that wave's lanes only (its tile
        // and pads are its own), and nothing writes the shared twiddle table again
        // unless the pass goes on to a fused inverse.
        if constexpr (kRowInWave && !FUSE) wave_lds_sync();
        else __syncthreads();
        if constexpr (KM > 0) {
          round_k<Pol, N_LOG, KM, false>(KL, t, TPT, tws, twg, m, lio, lio);
          __syncthreads();
        }
        if constexpr (FUSE) {
          // The low round's words stay thread-private from the forward stages through
          // the product and the inverse low round, so they go back to their own tile
          // places with no barrier; the inverse table and high factors replace the
          // forward ones (read only before the barrier above) meanwhile.
          TwStage<Pol, N, kTwMem> stage_i;
          stage_i.nthr = nthr;
          stage_i.load(twg_i);
          hi_load_from(edge_i.tt);
          if constexpr (kFoldI) {  // the thread's low factor of the inverse (its loads start here)
            const uint32_t lo = (uint32_t)t & ((1u << SIGMA) - 1);
            fold_i.a = buf_load_tw<Pol>(edge_i.tt, edge_i.tt_off + lo * kTw, 0);
            fold_i.aw = buf_load_tw<Pol>(edge_i.tt, edge_i.tt_off + ((1u << SIGMA) + (1u << (N_LOG - SIGMA)) + lo) * kTw, 0);
          }
          round_k<Pol, N_LOG, KL, true, false, LdsIO<false>, LdsIO<false>, NoHook, NoFold, false>(
              0, t, TPT, tws, twg, m, lio, lio, NoHook{}, NoFold{}, fmid);
          stage_i.store(tw_lds, twg_i);
          hi_store();
          __syncthreads();  // product tile, inverse table and inverse high factors complete
          if constexpr (KM > 0) {
            round_k<Pol, N_LOG, KM, false, false, LdsIO<false>, LdsIO<false>, NoHook, NoFold, true>(
                KL, t, TPT, tws, twg_i, m, lio, lio);
            __syncthreads();
          }
          round_k<Pol, N_LOG, KH, false, false, LdsIO<false>, decltype(gio_a), NoHook, decltype(fold_i), true>(
              KM + KL, t, TPT, tws, twg_i, m, lio, gio_a, NoHook{}, fold_i);
        } else if constexpr (Cols) {
          // the forward column pass is always the first of two: its output is never
          // reduced (the launcher rejects the flag)
          round_k<Pol, N_LOG, KL, true>(0, t, TPT, tws, twg, m, lio, gio.template with_out<kOutRaw>());
        } else {
          // Rows: a thread's low-round outputs are 2^KL consecutive words, so direct
          // stores would put neighbouring lanes 2^KL words apart.  Stage them in LDS
          // and write the tile out with consecutive lanes on consecutive 16 bytes.
          round_k<Pol, N_LOG, KL, true>(0, t, TPT, tws, twg, m, lio, lio);
          if constexpr (kRowInWave) wave_lds_sync();
          else __syncthreads();
          // (every thread moves kPer vectors of its row; the partner words of the fused
          // product are all requested before the first is used)
          constexpr int kPitch = kPitchT;
          constexpr int kChunks = N / kVec;
          constexpr int kPer = kChunks / TPT;
          static_assert(kPer * TPT == kChunks, "copy-out covers the tile exactly");
          const size_t tile0 = (size_t)unit * G * N;
          const auto ed = edge.template with_out<kOutCond>();
          // each thread moves chunks t + j TPT of its own row g
          Vec16 o[kPer];
#pragma unroll
          for (int j = 0; j < kPer; ++j) {
            const int c = copyout_row_chunk<kChunks, TPT>(t, j, g) * kVec;
            const Vec16 q = *reinterpret_cast<const Vec16 *>(tile + g * kPitch + c + ((c >> 5) << 2));
            const T *w = reinterpret_cast<const T *>(&q);
            T *wo = reinterpret_cast<T *>(&o[j]);
#pragma unroll
            for (int e = 0; e < kVec; ++e) wo[e] = ed.out(w[e], c + e);
          }
          HNTT_GLOBAL T *const out0 = (gio.pm ? gio.pm : gbase) + tile0;
          if (gio.pm) {  // fused pointwise product into the partner transform
            Vec16 pa[kPer];
#pragma unroll
            for (int j = 0; j < kPer; ++j)
              pa[j] = *reinterpret_cast<const HNTT_GLOBAL Vec16 *>(out0 + (size_t)g * N +
                                                                    copyout_row_chunk<kChunks, TPT>(t, j, g) * kVec);
#pragma unroll
            for (int j = 0; j < kPer; ++j) {
              const T *pw = reinterpret_cast<const T *>(&pa[j]);
              T *wo = reinterpret_cast<T *>(&o[j]);
#pragma unroll
              for (int e = 0; e < kVec; ++e) wo[e] = pmul_word<Pol>(wo[e], pw[e], m);
            }
          }
#pragma unroll
          for (int j = 0; j < kPer; ++j)
            *reinterpret_cast<HNTT_GLOBAL Vec16 *>(out0 + (size_t)g * N + copyout_row_chunk<kChunks, TPT>(t, j, g) * kVec) =
                o[j];
        }
      } else {
        round_k<Pol, N_LOG, KL, true>(0, t, TPT, tws, twg, m, gio, lio);
        stage.store(tw_lds, twg);
        hi_store();
        __syncthreads();  // tile, twiddle table and high factors complete
        if constexpr (KM > 0) {
          round_k<Pol, N_LOG, KM, false>(KL, t, TPT, tws, twg, m, lio, lio);
          __syncthreads();
        }
        const auto last = [&](const auto &dst) {
          round_k<Pol, N_LOG, KH, false>(KM + KL, t, TPT, tws, twg, m, lio, dst, NoHook{}, fold);
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

template <int Pol, bool Cols, int KH, int KM, int KL, bool TT, bool FUSE>
hipError_t launch_k(const KernelArgs &a, int blocks, int threads, size_t lds, hipStream_t stream) {
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_pass<Pol, Cols, KH, KM, KL, TT, FUSE>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  hipLaunchKernelGGL((k_pass<Pol, Cols, KH, KM, KL, TT, FUSE>), dim3(blocks), dim3(threads), lds, stream, a);
  return hipGetLastError();
}

// The fused product-and-inverse pass exists for 32-bit forward rows and whole
// transforms with the Shoup policies (the polynomial product's).
template <int Pol, bool Cols>
constexpr bool can_fuse() {
  return HNTT_WORD == 32 && !kInverse && !Cols && Pol != kPolicyMont;
}

// The split twiddle exists only in the row pass of a split transform (both directions).
template <int Pol, bool Cols, int KH, int KM, int KL>
hipError_t launch_tt(bool tt, bool fuse, const KernelArgs &a, int blocks, int threads, size_t lds,
                     hipStream_t stream) {
  if constexpr (can_fuse<Pol, Cols>()) {
    if (fuse)
      return tt ? launch_k<Pol, Cols, KH, KM, KL, true, true>(a, blocks, threads, lds, stream)
                : launch_k<Pol, Cols, KH, KM, KL, false, true>(a, blocks, threads, lds, stream);
  } else if (fuse) {
    return hipErrorInvalidValue;
  }
  if constexpr (Cols) {
    (void)tt;
    return launch_k<Pol, Cols, KH, KM, KL, false, false>(a, blocks, threads, lds, stream);
  } else {
    return tt ? launch_k<Pol, Cols, KH, KM, KL, true, false>(a, blocks, threads, lds, stream)
              : launch_k<Pol, Cols, KH, KM, KL, false, false>(a, blocks, threads, lds, stream);
  }
}

// Round splits per word size; must agree with pass_split().
template <int Pol, bool Cols>
hipError_t dispatch_n(int n, bool whole, bool tt, bool fuse, const KernelArgs &a, int blocks, int threads, size_t lds,
                      hipStream_t s) {
#define HNTT_CASE(N, KH, KM, KL) \
  case N: return launch_tt<Pol, Cols, KH, KM, KL>(tt, fuse, a, blocks, threads, lds, s);
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
  a.scale = (pp.kind == PassKind::kWhole && (pp.inverse || pp.fuse_inverse)) ? 1 : 0;
  if (pp.fuse_inverse) {
    // forward row or whole pass of a batch of products; the inverse output it writes
    // is final (whole: reduced) or the input of the inverse column pass (rows: raw)
    if (!pp.pm_off || pp.inverse || pp.kind == PassKind::kCols || !pp.table || pp.policy == kPolicyMont ||
        pp.normalize != (pp.kind == PassKind::kWhole))
      return hipErrorInvalidValue;
  } else if (pp.pm_off && (pp.inverse || pp.kind == PassKind::kCols || !pp.normalize)) {
    // the fused product belongs to the final forward pass (rows or whole) only
    return hipErrorInvalidValue;
  }
  if (pp.kind == PassKind::kCols && !pp.inverse && pp.normalize) return hipErrorInvalidValue;
  a.pm_off = pp.pm_off;
  if (pp.zero_upper && (pp.inverse || pp.kind == PassKind::kRows)) return hipErrorInvalidValue;
  a.zero_upper = pp.zero_upper ? 1 : 0;
  if (pp.table) {
    for (int i = 0; i < pp.nslots; ++i) a.slots[i] = pp.slots[i];
  } else {
    a.slots[0] = SlotParams{pp.p, pp.tw, pp.tt, pp.scale_w, pp.scale_wp, pp.jinv, nullptr, nullptr};
  }
  const int blocks = (int)total;
  using namespace HNTT_NS;
  const bool tt = pp.table ? pp.slots[0].tt != nullptr : pp.tt != nullptr;
  // a row pass applies the split twiddle and a whole-transform pass does not: the
  // kernel's table placement (and the LDS size above) relies on it
  if (!cols && tt != (pp.kind == PassKind::kRows)) return hipErrorInvalidValue;
  const bool fuse = pp.fuse_inverse;
  switch (pp.policy) {
    case kPolicyLazy:
      return cols ? dispatch_n<kPolicyLazy, true>(n, whole, tt, fuse, a, blocks, threads, lds, stream)
                  : dispatch_n<kPolicyLazy, false>(n, whole, tt, fuse, a, blocks, threads, lds, stream);
    case kPolicyPlain:
      return cols ? dispatch_n<kPolicyPlain, true>(n, whole, tt, fuse, a, blocks, threads, lds, stream)
                  : dispatch_n<kPolicyPlain, false>(n, whole, tt, fuse, a, blocks, threads, lds, stream);
    case kPolicyMont:
      return cols ? dispatch_n<kPolicyMont, true>(n, whole, tt, fuse, a, blocks, threads, lds, stream)
                  : dispatch_n<kPolicyMont, false>(n, whole, tt, fuse, a, blocks, threads, lds, stream);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace hntt
