// Issue rates of the integer VALU instructions the butterflies are built from,
// the shader clock under load, and plain device-copy bandwidth, on the GPU this
// runs on.  Each rate kernel keeps eight independent dependency chains per lane
// (so latency is hidden) of exactly one instruction per step; the generated
// code of each loop body is that one instruction (checked in the gfx950
// assembly of this file).  Output: one line per measurement, then a JSON line.
//
//   usage: valu_rates [iters]
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <string>
#include <vector>

#define CHECK(x)                                                                      \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) {                                                           \
      fprintf(stderr, "%s:%d %s: %s\n", __FILE__, __LINE__, #x, hipGetErrorString(e_)); \
      exit(2);                                                                        \
    }                                                                                 \
  } while (0)

constexpr int kChains = 8;
constexpr int kThreads = 256;

enum Op { kAdd, kMulLo, kMulHi, kMad64, kAdd3, kXad, kNumOps };
static const char *kOpName[kNumOps] = {"v_add_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_mad_u64_u32",
                                       "v_add3_u32", "v_xad_u32"};

template <int OP>
__global__ void __launch_bounds__(kThreads) k_rate(uint32_t *out, uint32_t b, uint32_t c, int iters) {
  uint32_t a[kChains];
  uint64_t w[kChains];
  // operands kept in VGPRs: a VALU instruction may read at most one scalar register
  asm volatile("" : "+v"(b));
  asm volatile("" : "+v"(c));
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    a[j] = threadIdx.x * 2654435761u + j;
    w[j] = ((uint64_t)a[j] << 32) | (a[j] ^ c);
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
      if constexpr (OP == kAdd) a[j] = a[j] + b;
      else if constexpr (OP == kMulLo) a[j] = a[j] * b;
      else if constexpr (OP == kMulHi) a[j] = __umulhi(a[j], b);
      else if constexpr (OP == kMad64) w[j] = (uint64_t)(uint32_t)w[j ^ 1] * b + w[j];  // no dst/src overlap
      else if constexpr (OP == kAdd3) a[j] = a[j] + a[j ^ 1] + b;
      else a[j] = (a[j] ^ c) + b;  // kXad; c is ~0 at run time
    }
  }
  uint32_t r = 0;
#pragma unroll
  for (int j = 0; j < kChains; ++j) r ^= a[j] ^ (uint32_t)w[j] ^ (uint32_t)(w[j] >> 32);
  out[blockIdx.x * kThreads + threadIdx.x] = r;
}

// Shader-clock ticks (s_memtime) against the constant 100 MHz counter (s_memrealtime)
// over a long dependent loop, one record per workgroup, with every CU busy.
__global__ void __launch_bounds__(kThreads) k_clock(uint64_t *rec, uint32_t b, int iters) {
  uint32_t a = threadIdx.x;
  const uint64_t c0 = clock64(), r0 = wall_clock64();
  for (int i = 0; i < iters; ++i) a = a * b + 1;
  const uint64_t c1 = clock64(), r1 = wall_clock64();
  if (threadIdx.x == 0) {
    rec[2 * blockIdx.x] = c1 - c0;
    rec[2 * blockIdx.x + 1] = (r1 - r0) | ((uint64_t)(a & 1) << 63);
  }
}

typedef uint32_t Vec4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(kThreads) k_copy(const Vec4 *__restrict__ src, Vec4 *__restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (size_t)gridDim.x * kThreads)
    dst[i] = src[i];
}

template <class F>
static float time_ms(F launch, int reps) {
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  float best = 1e30f;
  for (int r = 0; r < reps; ++r) {
    CHECK(hipEventRecord(e0, 0));
    launch();
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    best = std::min(best, ms);
  }
  CHECK(hipEventDestroy(e0));
  CHECK(hipEventDestroy(e1));
  return best;
}

template <int OP>
static float run_rate(uint32_t *out, int blocks, int iters) {
  return time_ms([&] { hipLaunchKernelGGL(k_rate<OP>, dim3(blocks), dim3(kThreads), 0, 0, out, 2654435761u, ~0u, iters); },
                 5);
}

int main(int argc, char **argv) {
  const int iters = argc > 1 ? atoi(argv[1]) : 4096;
  hipDeviceProp_t prop;
  CHECK(hipGetDeviceProperties(&prop, 0));
  const int cus = prop.multiProcessorCount;
  const double nominal_ghz = 2.4;
  printf("device %s, %d CUs, clockRate %.0f MHz (reported)\n", prop.gcnArchName, cus, prop.clockRate / 1e3);
  const int blocks = cus * 8;  // 8 workgroups of 4 waves per CU: 8 waves per SIMD
  uint32_t *out = nullptr;
  CHECK(hipMalloc(&out, (size_t)blocks * kThreads * sizeof(uint32_t)));
  // warm the clocks
  for (int i = 0; i < 20; ++i) hipLaunchKernelGGL(k_rate<kAdd>, dim3(blocks), dim3(kThreads), 0, 0, out, 3u, ~0u, iters);
  CHECK(hipDeviceSynchronize());

  float ms[kNumOps];
  ms[kAdd] = run_rate<kAdd>(out, blocks, iters);
  ms[kMulLo] = run_rate<kMulLo>(out, blocks, iters);
  ms[kMulHi] = run_rate<kMulHi>(out, blocks, iters);
  ms[kMad64] = run_rate<kMad64>(out, blocks, iters);
  ms[kAdd3] = run_rate<kAdd3>(out, blocks, iters);
  ms[kXad] = run_rate<kXad>(out, blocks, iters);
  const double wave_insts = (double)blocks * (kThreads / 64) * iters * kChains;

  // loaded shader clock
  uint64_t *rec = nullptr;
  CHECK(hipMalloc(&rec, (size_t)blocks * 2 * sizeof(uint64_t)));
  hipLaunchKernelGGL(k_clock, dim3(blocks), dim3(kThreads), 0, 0, rec, 2654435761u, iters * 64);
  CHECK(hipDeviceSynchronize());
  std::vector<uint64_t> hrec((size_t)blocks * 2);
  CHECK(hipMemcpy(hrec.data(), rec, hrec.size() * sizeof(uint64_t), hipMemcpyDeviceToHost));
  std::vector<double> mhz;
  for (int i = 0; i < blocks; ++i) {
    const double ticks = (double)hrec[2 * i], real = (double)(hrec[2 * i + 1] & ~(1ull << 63));
    if (real > 0) mhz.push_back(ticks / real * 100.0);  // s_memrealtime runs at 100 MHz
  }
  std::sort(mhz.begin(), mhz.end());
  const double clock_mhz = mhz.empty() ? 0 : mhz[mhz.size() / 2];

  // device copy, 1 GiB each way
  const size_t bytes = (size_t)1 << 30, n = bytes / sizeof(Vec4);
  Vec4 *src = nullptr, *dst = nullptr;
  CHECK(hipMalloc(&src, bytes));
  CHECK(hipMalloc(&dst, bytes));
  CHECK(hipMemset(src, 1, bytes));
  const float copy_ms = time_ms([&] { hipLaunchKernelGGL(k_copy, dim3(cus * 64), dim3(kThreads), 0, 0, src, dst, n); }, 10);
  const double copy_gbs = 2.0 * bytes / (copy_ms * 1e-3) / 1e9;

  printf("%-16s %10s %14s %14s %14s\n", "instruction", "ms", "Gwave-inst/s", "per CU/2.4GHz", "per CU/clock");
  std::string json = "{\"cus\": " + std::to_string(cus) + ", \"clock_mhz_loaded\": " + std::to_string(clock_mhz) +
                     ", \"copy_GBs\": " + std::to_string(copy_gbs) + ", \"rates\": {";
  for (int o = 0; o < kNumOps; ++o) {
    const double rate = wave_insts / (ms[o] * 1e-3);
    const double per_nom = rate / (cus * nominal_ghz * 1e9);
    const double per_clk = clock_mhz > 0 ? rate / (cus * clock_mhz * 1e6) : 0;
    printf("%-16s %10.3f %14.1f %14.3f %14.3f\n", kOpName[o], ms[o], rate / 1e9, per_nom, per_clk);
    json += std::string(o ? ", " : "") + "\"" + kOpName[o] + "\": " + std::to_string(per_clk);
  }
  printf("shader clock under load (median of %zu workgroups): %.0f MHz\n", mhz.size(), clock_mhz);
  printf("device copy 1 GiB: %.3f ms, %.0f GB/s (read + write)\n", copy_ms, copy_gbs);
  json += "}, \"unit\": \"wave64 instructions per CU per shader clock\"}";
  printf("%s\n", json.c_str());
  CHECK(hipFree(out));
  CHECK(hipFree(rec));
  CHECK(hipFree(src));
  CHECK(hipFree(dst));
  return 0;
}
