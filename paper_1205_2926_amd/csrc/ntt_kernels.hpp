// Host-visible launch interface of the NTT pass kernels (ntt_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hntt {

constexpr int kMaxBatchPerLaunch = 64;

// Device pointers of the transforms one launch works on, passed by value.
struct BatchPtrs {
  uint64_t ptr[kMaxBatchPerLaunch];
};

// A transform listed in a device-side table (batched polynomial products): its data
// pointer and the slot of its prime in the launch's PassParams::slots.
struct XformEntry {
  uint64_t ptr;
  uint32_t slot;
  uint32_t reserved;
};

constexpr int kMaxSlots = 4;

// Butterfly policy of a launch.
enum : int {
  kPolicyPlain = 0,  // Algorithm 2 and the fully reducing inverse (Shoup products)
  kPolicyLazy = 1,   // Algorithms 3 and 4 (Shoup products, W and W' = floor(W beta / p))
  kPolicyMont = 2,   // Algorithm 5 and its inverse (Montgomery products, W' = W beta mod p only)
};

// Per-prime launch parameters (tables built for the launch's sub-transform length).
// Table entries are (W, W') pairs for the Shoup policies and single words
// W beta mod p for the Montgomery policy.
struct SlotParams {
  uint64_t p;
  const void *tw;     // per-stage twiddles of omega_N^(+-j)
  const void *tt;     // split-twiddle factors of the pass (null when it has none)
  uint64_t scale_w;   // kWhole inverse: L^-1 (Montgomery policy: L^-1 beta mod p)
  uint64_t scale_wp;  // and its Shoup constant (unused by the Montgomery policy)
  uint64_t jinv;      // p^-1 mod beta (Montgomery policy; fused pointwise product)
  // fused forward + inverse launch (PassParams::fuse_inverse): the inverse
  // transform's per-stage table and split-twiddle factors of the same sub-transform
  const void *tw2;
  const void *tt2;
};

// Which pass of the transform a launch performs.
enum class PassKind : int {
  kWhole = 0,  // the whole transform of length 2^n inside one workgroup
  kRows = 1,   // contiguous rows of length 2^n (innermost stages)
  kCols = 2,   // strided columns of length 2^n (outermost stages) plus the split twiddle
};

constexpr int kMaxPassLog = 12;      // longest sub-transform inside one workgroup: 2^12 words
constexpr int kMaxPassThreads = 512; // workgroup size limit of the pass kernels (keeps 256 VGPRs available)

// Register rounds of a sub-transform of 2^n words: bits of the high, middle and
// low rounds (KH + KM + KL = n; KH = 0 means a single round of n bits, KM = 0
// two rounds).  A thread holds 2^K words of a round in registers; 64-bit words
// use smaller rounds to stay within the register file.
struct RoundSplit {
  int kh, km, kl;
};
// `whole`: a one-pass transform, one per workgroup; 2^9 and 2^10 u32 words then
// use three rounds so that the transform has a full wave of 64 threads (two
// rounds would give it 32, half of every wave idle).
inline RoundSplit pass_split(int n, int word_bits, bool whole = false) {
  if (word_bits == 32) {
    if (whole && n == 9) return {3, 3, 3};
    if (whole && n == 10) return {4, 3, 3};
    if (n <= 6) return {0, 0, n};
    if (n <= 10) return {(n + 1) / 2, 0, n / 2};
    // n = 11, 12: three rounds of at most 16 words per thread, so that a 2^n-word
    // tile has enough threads to fill the CU that its LDS footprint allows
    return {4, 4, n - 8};
  }
  if (n <= 5) return {0, 0, n};
  if (n <= 8) return {(n + 1) / 2, 0, n / 2};
  if (n == 9) return {3, 3, 3};
  if (n == 10) return {4, 3, 3};
  return {4, 4, n - 8};
}
// Row tiles in LDS: four pad words after every 32 words of a row, so that
// consecutive threads of the low round (16-byte vector accesses, 2^KL words
// apart) fall in distinct banks.  (One pad per 64 words instead, which would
// also spare the copy out of the tile its few two-way conflicts, put conflicts
// into the low round: three times the conflict cycles, measured.)
constexpr size_t row_padded_len(size_t N) { return N + (N >> 5) * 4; }
// Extra words between consecutive row tiles of 32-bit words when a row has fewer
// than 32 threads (TPT = 2^(n - largest round)): the 32-bit LDS accesses of one
// half-wave (32 lanes, 32 banks) then cover several rows, and shifting each row
// by TPT words puts their lanes on disjoint banks (the padded pitch alone is a
// multiple of 32 words).
constexpr size_t row_skew(int n, int kh, int km, int kl, int word_bits) {
  const int kmax = kh > km ? (kh > kl ? kh : kl) : (km > kl ? km : kl);
  const int tpt = 1 << (n - kmax);
  return (word_bits == 32 && kh > 0 && tpt < 32) ? (size_t)tpt : 0;
}

// Whether the rounds of a pass over 2^n-word sub-transforms that do not have
// compile-time twiddles read them from global memory (L1/L2) instead of an LDS
// copy of the table.  For 64-bit words the copy (16-byte entries: a third of
// the LDS next to a 2^11-word tile) would cost a workgroup per CU.  For 32-bit
// words, forward passes over rows or whole transforms (fwd) read from memory at
// 2^10 words: without the 8 KB copy four workgroups of eight rows fit a CU
// instead of three, and the staging registers are freed (2^10-word rows: 114
// against 124 us per 64 x 2^20 launch).  Above 2^10 words only whole transforms
// (whole) do: the product batch's 2^11- and 2^12-word transforms ran 4% faster
// from memory, the large-integer batch's 2^11-word rows 2% slower.  The column
// passes and the inverse passes keep the copy (from memory they ran 9-16%
// slower), and so do shorter forward passes (the product batch's 2^6- to
// 2^9-word passes ran 4-6% slower from memory).
constexpr bool tw_global(int n, int word_bits, bool fwd, bool whole) {
  return word_bits == 64 || (fwd && (n == 10 || (n > 10 && whole)));
}

// Threads per sub-transform: one group of the largest round each.
inline int pass_tpt(int n, int word_bits, bool whole = false) {
  const RoundSplit r = pass_split(n, word_bits, whole);
  const int kmax = r.kh > r.kl ? (r.kh > r.km ? r.kh : r.km) : (r.kl > r.km ? r.kl : r.km);
  return 1 << (n - kmax);
}

struct PassParams {
  PassKind kind;
  int word_bits;   // 32 or 64
  int policy;      // kPolicyPlain, kPolicyLazy or kPolicyMont
  bool inverse;    // Algorithm 1 forward (false) or run backwards (true)
  bool normalize;  // reduce the final output to [0,p)
  int n;           // log2 of the sub-transform length handled inside a workgroup
  int log_other;   // kRows: log2(#rows) ; kCols: log2(#columns) ; kWhole: 0
  int group;       // sub-transforms per workgroup
  int nbatch;      // transforms in this launch (<= kMaxBatchPerLaunch unless `table` is set)
  uint64_t p;
  const void *tw;     // per-stage twiddle table of the sub-transform (heap order)
  const void *tt;     // split-twiddle factors of the second pass of a transform, else null
  uint64_t scale_w;   // kWhole inverse: L^-1 (Montgomery policy: L^-1 beta mod p)
  uint64_t scale_wp;  // and its Shoup constant
  uint64_t jinv;      // Montgomery policy: p^-1 mod beta
  // Final forward pass only: when nonzero, every output word is multiplied by the
  // word at the same position of the "partner" transform that starts pm_off words
  // before this one, and the product replaces the partner's word (this transform's
  // own words are left stale).  Used by the polynomial product: B_k's last pass
  // multiplies into A_k.  The partner's words must be fully reduced and carry a
  // factor beta (its operand was prepared times beta mod p): the product is one
  // Montgomery product, in [0,2p) (lazy policy) or [0,p) (plain), the input range
  // of the inverse transform that follows.
  uint32_t pm_off;
  // With pm_off, 32-bit words, a table and a Shoup policy only: instead of writing
  // the product, run the inverse transform's row pass (kRows) or whole transform
  // (kWhole, times L^-1 and fully reduced when normalize is set) on it and write
  // that over the partner (slots' tw2/tt2 tables).  The inverse row output is left
  // in the range the following inverse column pass accepts.
  bool fuse_inverse;
  // First forward pass only: the upper half of every input (positions >= 2^l / 2)
  // is known to be zero, so it is not read (the padded operands of a product).
  bool zero_upper;
  // Batched form: transforms listed in a device table, each with its prime's slot;
  // when `table` is set, p/tw/tt/scale above are ignored and slots[] is used.
  const XformEntry *table;
  int nslots;
  SlotParams slots[kMaxSlots];
};

hipError_t launch_pass_u32_fwd(const PassParams &pp, const BatchPtrs &ptrs, hipStream_t stream);
hipError_t launch_pass_u32_inv(const PassParams &pp, const BatchPtrs &ptrs, hipStream_t stream);
hipError_t launch_pass_u64_fwd(const PassParams &pp, const BatchPtrs &ptrs, hipStream_t stream);
hipError_t launch_pass_u64_inv(const PassParams &pp, const BatchPtrs &ptrs, hipStream_t stream);

// Enqueue one pass over `ptrs` on `stream`.  Returns a hipError_t.
hipError_t launch_pass(const PassParams &pp, const BatchPtrs &ptrs, hipStream_t stream);

// Butterfly unit-test kernel launcher (kind as in hntt_debug_butterfly).
hipError_t launch_debug_butterfly(int kind, int word_bits, uint64_t p, const void *x, const void *y,
                                  const void *w, const void *wp, void *xo, void *yo, size_t n,
                                  hipStream_t stream);

// Pointwise product c = a b mod p over len words.
hipError_t launch_pointwise(int word_bits, uint64_t p, const void *a, const void *b, void *c, uint64_t len,
                            hipStream_t stream);

// LDS bytes a pass needs (0 if it cannot run).
size_t pass_lds_bytes(const PassParams &pp);

}  // namespace hntt
