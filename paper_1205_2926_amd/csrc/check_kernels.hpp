// Device-side input checks behind the HNTT_VALIDATE flag.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace hntt {

// *flag = value, written by a one-thread kernel on `stream`.
hipError_t launch_set_flag(uint32_t *flag, uint32_t value, hipStream_t stream);

// If any of the `len` words (word_bits 32 or 64) at x is >= bound, lower *first_bad to `index`
// (an atomic minimum, so that over several launches the flag ends at the smallest index with
// an out-of-range word).
hipError_t launch_range_check(int word_bits, const void *x, uint64_t len, uint64_t bound, uint32_t index,
                              uint32_t *first_bad, hipStream_t stream);

}  // namespace hntt
