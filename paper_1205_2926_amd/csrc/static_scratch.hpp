// Static device workspace of the allocation-free product entry point.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "hntt.h"

namespace hntt {

constexpr size_t kStaticScratchBytes = HNTT_STATIC_SCRATCH_BYTES;
constexpr int kStaticScratchMaxDevices = 64;

// Device address of the static workspace on `device`, which must be the current
// device.  Looked up with hipGetSymbolAddress on the first call per device and
// cached; thread-safe.
hipError_t static_scratch_address(int device, void **out);

}  // namespace hntt
