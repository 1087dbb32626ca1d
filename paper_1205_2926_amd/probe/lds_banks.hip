// How the LDS serves the lanes of a wave on the GPU this runs on: in each test only
// two lanes (a, b) are active and access LDS at word offsets 0 and `off`, 256 times
// per wave; the bank-conflict counter of the dispatch (rocprofv3 --pmc
// SQ_LDS_BANK_CONFLICT SQ_WAVES) then says whether the two lanes are served in the
// same cycle (a conflict needs that) and whether the two offsets share a bank.
// Accesses: 32-bit reads, 16-byte reads and 16-byte writes.  One line per test is
// printed before its launch; every address lies inside the 64 KiB array.
//
//   usage: lds_banks
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#define CHECK(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_)); exit(2);} } while (0)
constexpr int kWords = 16384;
constexpr int kIters = 256;
typedef uint32_t V4 __attribute__((ext_vector_type(4)));
// MODE 0: b32 read, 2: b128 read, 3: b128 write
template <int MODE>
__global__ void __launch_bounds__(64) k_pair(int la, int lb, int off, uint32_t *out) {
  __shared__ V4 lds4[kWords / 4];
  uint32_t *lds = reinterpret_cast<uint32_t *>(lds4);
  const int lane = threadIdx.x;
  for (int i = lane; i < kWords; i += 64) lds[i] = i * 2654435761u;
  __syncthreads();
  uint32_t acc = 0;
  V4 vacc = {0, 0, 0, 0};
  if (lane == la || lane == lb) {
    int ad = lane == la ? 0 : off;
    for (int it = 0; it < kIters; ++it) {
      asm volatile("" : "+v"(ad));
      if constexpr (MODE == 0) acc += lds[ad];
      else if constexpr (MODE == 2) vacc += lds4[ad >> 2];
      else { V4 v = {(uint32_t)it, acc, 1u, 2u}; lds4[ad >> 2] = v; }
    }
  }
  __syncthreads();
  out[blockIdx.x * 64 + lane] = acc + vacc.x + vacc.y + vacc.z + vacc.w + lds[lane];
}
int main() {
  uint32_t *dout;
  CHECK(hipMalloc(&dout, 64 * 64 * sizeof(uint32_t)));
  struct T { int mode, la, lb, off; };
  T tests[2048]; int n = 0;
  // b128 read: lane 0 (and lane 5) against every other lane at a same-bank offset
  for (int base : {0, 5, 40})
    for (int j = 0; j < 64; ++j) if (j != base) tests[n++] = {2, base, j, 1024};
  // b128 read: bank count, lane 0 against lanes 1..63 at offsets 32, 64
  for (int off : {32, 64})
    for (int j = 1; j < 64; ++j) tests[n++] = {2, 0, j, off};
  // b128 write: lane 0 against every other lane
  for (int j = 1; j < 64; ++j) tests[n++] = {3, 0, j, 1024};
  // b32 read: lane 0 against every other lane, offsets 1024 and 32
  for (int off : {1024, 32})
    for (int j = 1; j < 64; ++j) tests[n++] = {0, 0, j, off};
  for (int i = 0; i < n; ++i) {
    const T &t = tests[i];
    if (t.off < 0 || t.off + 4 > kWords || t.off % 4) return 1;
    printf("test mode %d lanes %d %d off %d\n", t.mode, t.la, t.lb, t.off);
    if (t.mode == 0) hipLaunchKernelGGL(k_pair<0>, dim3(64), dim3(64), 0, 0, t.la, t.lb, t.off, dout);
    else if (t.mode == 2) hipLaunchKernelGGL(k_pair<2>, dim3(64), dim3(64), 0, 0, t.la, t.lb, t.off, dout);
    else hipLaunchKernelGGL(k_pair<3>, dim3(64), dim3(64), 0, 0, t.la, t.lb, t.off, dout);
  }
  CHECK(hipDeviceSynchronize());
  printf("done %d\n", n);
  return 0;
}
