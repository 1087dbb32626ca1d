// Device workspace of hntt_polymul_crt_static: one file-scope array that every
// GPU the library is loaded on holds until the process ends.  Host code never
// passes the array's name to a kernel or a copy (on the host it names a
// stand-in, not device memory); it asks for the array's device address once per
// GPU, with that GPU current, and uses that address everywhere.
#include <hip/hip_runtime.h>

#include <mutex>

#include "static_scratch.hpp"

namespace hntt {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_addr[kStaticScratchMaxDevices];
}  // namespace

hipError_t static_scratch_address(int device, void **out) {
  if (device < 0 || device >= kStaticScratchMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;  // the caller makes `device` current first
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[device] = p;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

}  // namespace hntt
