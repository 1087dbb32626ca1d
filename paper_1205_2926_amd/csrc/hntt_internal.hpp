// Internal state of a library context (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <functional>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "hntt.h"

namespace hntt {

struct DeviceBuffer {
  void *ptr = nullptr;
  size_t bytes = 0;
  DeviceBuffer() = default;
  DeviceBuffer(const DeviceBuffer &) = delete;
  DeviceBuffer &operator=(const DeviceBuffer &) = delete;
  ~DeviceBuffer();
};

// How a transform of length 2^l is split into passes.
struct Plan {
  bool split;  // false: one whole-transform pass
  int r;       // log2 of the column-transform length (split) or l (whole)
  int c;       // log2 of the row length (split)
  int g_cols;  // columns per workgroup in the column pass
  int g_rows;  // rows per workgroup in the row pass (forward; polynomial products)
  int g_rows_inv;  // rows per workgroup in the inverse transform's row pass
  int chunk;   // transforms per launch; every pass runs on one chunk before the next chunk
};

// Device twiddle tables for one (p, omega, l, word_bits, form): arrays of
// interleaved (W, W') pairs with W' = floor(W beta / p) (Shoup form), or of
// single words W beta mod p (Montgomery form).
struct Tables {
  Plan plan;
  bool mont;                             // Montgomery-form tables (single words W beta mod p)
  uint64_t linv, linv_p;                 // L^-1 mod p and its Shoup constant (Montgomery: L^-1 beta mod p, 0)
  uint64_t jinv;                         // p^-1 mod beta
  const void *fwd, *inv;                 // whole transform, or the column transform
  const void *row_fwd, *row_inv;         // row transform (split)
  const void *tt_fwd, *tt_inv;           // split twiddles (split)
};

}  // namespace hntt

namespace hntt {
struct TraceEvent {
  std::string name;
  hipEvent_t start, stop;
};
struct TraceAcc {
  uint64_t launches = 0;
  double total_ms = 0;
};
}  // namespace hntt

struct hntt_polymul_plan;

struct hntt_ctx {
  int device = 0;
  size_t budget = 0;
  size_t bytes_held = 0;
  bool device_ready = false;
  std::string last_error;
  std::map<uint64_t, bool> prime_cache;
  // (p, omega, l, word bits, Montgomery form, row-pass length c) -> resident tables
  std::map<std::tuple<uint64_t, uint64_t, int, int, bool, int>, hntt::Tables> tables;
  std::map<std::pair<int, int>, hntt_tuning> tuning;  // (log2_len, word_bits) -> schedule override
  std::vector<std::unique_ptr<hntt::DeviceBuffer>> buffers;
  hntt_polymul_plan *poly_cache = nullptr;  // last plan of hntt_polymul_crt
  std::vector<unsigned char> static_meta;    // host image of the last hntt_polymul_crt_static metadata
  uint32_t *check_flag = nullptr;            // device word for HNTT_VALIDATE (allocated on first use)
  void release_poly_cache();
  bool trace = false;
  std::vector<hntt::TraceEvent> trace_pending;
  std::map<std::string, hntt::TraceAcc> trace_acc;
  void release_device_state() {
    tables.clear();
    if (check_flag) (void)hipFree(check_flag);
    check_flag = nullptr;
    for (auto &ev : trace_pending) {
      (void)hipEventDestroy(ev.start);
      (void)hipEventDestroy(ev.stop);
    }
    trace_pending.clear();
  }
};

namespace hntt {
int check_desc(hntt_ctx *ctx, const hntt_desc &d, uint32_t flags);
// row_log2: the row pass's stages (0: the built-in ceil(l / 2)).
Plan make_plan(int l, int word_bits, int row_log2 = 0);
Plan effective_plan(const hntt_ctx *ctx, int l, int word_bits);
int check_tuning(const hntt_tuning &t, std::string *why);
int ensure_device(hntt_ctx *ctx);
// Tables for the split of make_plan(l, bits, row_log2).
int get_tables(hntt_ctx *ctx, uint64_t p, uint64_t omega, int l, int bits, bool mont, int row_log2,
               const Tables **out);
// The resident tables of (p, omega, l, bits, form), or null; builds nothing.
const Tables *find_tables(const hntt_ctx *ctx, uint64_t p, uint64_t omega, int l, int bits, bool mont, int row_log2);
// Launch wrappers that record HIP events around the launch when tracing is on
// (hntt_trace_*): any launch under a kernel name, or one NTT pass under its name.
struct PassParams;
struct BatchPtrs;
hipError_t trace_launch(hntt_ctx *ctx, const std::string &name, hipStream_t stream,
                        const std::function<hipError_t()> &launch);
hipError_t launch_traced(hntt_ctx *ctx, const PassParams &pp, const BatchPtrs &bp, hipStream_t stream);
int transform(hntt_ctx *ctx, const hntt_desc *descs, size_t n, uint32_t flags, void *stream, bool inverse);
}  // namespace hntt
