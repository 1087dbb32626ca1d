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

// Which pass of the transform a launch performs.
enum class PassKind : int {
  kWhole = 0,  // the whole transform of length 2^n inside one workgroup
  kRows = 1,   // contiguous rows of length 2^n (innermost stages)
  kCols = 2,   // strided columns of length 2^n (outermost stages) plus the split twiddle
};

struct PassParams {
  PassKind kind;
  int word_bits;   // 32 or 64
  bool lazy;       // Algorithm 3/4 (true) or fully reducing (false)
  bool inverse;    // Algorithm 1 forward (false) or run backwards (true)
  bool normalize;  // reduce the final output to [0,p)
  int n;           // log2 of the sub-transform length handled inside a workgroup
  int log_other;   // kRows: log2(#rows) ; kCols: log2(#columns) ; kWhole: 0
  int group;       // sub-transforms per workgroup
  int nbatch;      // transforms in this launch (<= kMaxBatchPerLaunch)
  uint64_t p;
  const void *tw_w;   // table of omega_N^(+-j), j < 2^(n-1)
  const void *tw_wp;  // Shoup constants of tw_w
  const void *tt_w;   // kCols: split twiddles, same shape as the data
  const void *tt_wp;
  uint64_t scale_w;   // kWhole inverse: L^-1 and its Shoup constant
  uint64_t scale_wp;
};

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
