// C ABI of the library (include/hntt.h): argument checking, planning,
// twiddle-table cache and kernel dispatch.  Host code only; the kernels live
// in ntt_kernels.hip.
#include "hntt.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "check_kernels.hpp"
#include "hntt_internal.hpp"
#include "ntt_kernels.hpp"
#include "numtheory.hpp"

using namespace hntt;

namespace hntt {

// ------------------------------------------------------------------------------------------------
// Device buffers owned by the context.
DeviceBuffer::~DeviceBuffer() {
  if (ptr) (void)hipFree(ptr);
}

}  // namespace hntt

namespace {

int set_error(hntt_ctx *ctx, int status, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int set_error(hntt_ctx *ctx, int status, const char *fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return status;
}

int hip_status(hntt_ctx *ctx, hipError_t e, const char *what) {
  if (e == hipSuccess) return HNTT_OK;
  if (e == hipErrorOutOfMemory) return set_error(ctx, HNTT_ENOMEM, "%s: %s", what, hipGetErrorString(e));
  return set_error(ctx, HNTT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Restores the caller's current device on scope exit.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

bool prime_cached(hntt_ctx *ctx, uint64_t p) {
  auto it = ctx->prime_cache.find(p);
  if (it != ctx->prime_cache.end()) return it->second;
  const bool r = is_prime_u64(p);
  ctx->prime_cache[p] = r;
  return r;
}

int max_whole_log(int word_bits) { return word_bits == 32 ? 12 : 11; }

}  // namespace

namespace hntt {

int check_desc(hntt_ctx *ctx, const hntt_desc &d, uint32_t flags) {
  const bool plain = flags & HNTT_PLAIN;
  if (d.word_bits != 32 && d.word_bits != 64)
    return set_error(ctx, HNTT_EINVAL, "word_bits must be 32 or 64 (got %u)", d.word_bits);
  if (!d.data) return set_error(ctx, HNTT_EINVAL, "data pointer is NULL");
  if (d.log2_len < 1 || d.log2_len > 30)
    return set_error(ctx, HNTT_EINVAL, "log2_len must be in [1, 30] (got %u)", d.log2_len);
  {
    // 16-byte vector accesses: data aligned to 16 bytes or to its own size if smaller
    const uint64_t bytes = (uint64_t)(d.word_bits / 8) << d.log2_len;
    const uint64_t align = bytes < 16 ? bytes : 16;
    if (reinterpret_cast<uintptr_t>(d.data) % align)
      return set_error(ctx, HNTT_EINVAL, "data pointer is not aligned to %llu bytes", (unsigned long long)align);
  }
  if (d.p < 3 || !(d.p & 1)) return set_error(ctx, HNTT_EINVAL, "p must be an odd prime (got %llu)",
                                              (unsigned long long)d.p);
  const unsigned limit_bits = d.word_bits - (plain ? 1 : 2);  // p < beta/2 (Alg. 2) or beta/4 (Alg. 3, 4)
  if (limit_bits < 64 && d.p >= (1ull << limit_bits))
    return set_error(ctx, HNTT_EUNSUPPORTED, "p = %llu needs p < 2^%u for %s butterflies on %u-bit words",
                     (unsigned long long)d.p, limit_bits, plain ? "plain" : "lazy", d.word_bits);
  if ((d.p - 1) % (1ull << d.log2_len))
    return set_error(ctx, HNTT_EINVAL, "2^%u does not divide p - 1", d.log2_len);
  if (!prime_cached(ctx, d.p)) return set_error(ctx, HNTT_EINVAL, "p = %llu is not prime", (unsigned long long)d.p);
  if (d.omega == 0 || d.omega >= d.p)
    return set_error(ctx, HNTT_EINVAL, "omega must be in [1, p)");
  if (powmod(d.omega, 1ull << (d.log2_len - 1), d.p) != d.p - 1)
    return set_error(ctx, HNTT_EINVAL, "omega is not a primitive 2^%u-th root of unity mod p", d.log2_len);
  const int lmax = max_whole_log((int)d.word_bits);
  if ((int)d.log2_len > 2 * lmax)
    return set_error(ctx, HNTT_EUNSUPPORTED, "log2_len %u exceeds the two-pass limit %d for %u-bit words",
                     d.log2_len, 2 * lmax, d.word_bits);
  return HNTT_OK;
}

Plan make_plan(int l, int word_bits, int row_log2) {
  Plan pl{};
  const int lmax = max_whole_log(word_bits);
  if (l <= lmax) {
    pl.split = false;
    pl.r = l;
    pl.c = 0;
    pl.g_cols = pl.g_rows = pl.g_rows_inv = 1;
    return pl;
  }
  pl.split = true;
  pl.c = row_log2 ? row_log2 : (l + 1) / 2;
  pl.r = l - pl.c;
  // a group fits when both directions of its pass fit (the forward row pass may keep
  // no LDS copy of the twiddle table; the inverse one does)
  auto lds_ok = [&](PassKind kind, int n, int g) {
    if (pass_split(n, word_bits).kh == 0) return true;
    for (const bool inverse : {false, true}) {
      PassParams pp{};
      pp.kind = kind;
      pp.inverse = inverse;
      pp.word_bits = word_bits;
      pp.n = n;
      pp.group = g;
      const size_t b = pass_lds_bytes(pp);
      if (!b || b > 80 * 1024) return false;
    }
    return true;
  };
  // column pass: adjacent columns per workgroup so that each row segment is at least 64
  // bytes, and at least 256 threads when the column transforms are short
  int g = std::max(word_bits == 32 ? 16 : 8, 256 / pass_tpt(pl.r, word_bits));
  while (g > 1 && (pass_tpt(pl.r, word_bits) * g > kMaxPassThreads || g > (1 << pl.c) || !lds_ok(PassKind::kCols, pl.r, g)))
    g >>= 1;
  pl.g_cols = g;
  // row pass: up to 512 threads per workgroup (the fastest row-pass shape measured at L = 2^20)
  int gr = std::max(1, kMaxPassThreads / pass_tpt(pl.c, word_bits));
  while (gr > 1 && (gr > (1 << pl.r) || !lds_ok(PassKind::kRows, pl.c, gr))) gr >>= 1;
  pl.g_rows = pl.g_rows_inv = gr;
  pl.chunk = kMaxBatchPerLaunch;
  return pl;
}

// A schedule override is legal when every pass fits the kernels' limits.
int check_tuning(const hntt_tuning &t, std::string *why) {
  auto fail = [&](const char *m) {
    if (why) *why = m;
    return HNTT_EINVAL;
  };
  if (t.word_bits != 32 && t.word_bits != 64) return fail("word_bits must be 32 or 64");
  const int lmax = max_whole_log((int)t.word_bits);
  if (t.log2_len < 1 || (int)t.log2_len > 2 * lmax) return fail("log2_len outside the two-pass range");
  if (t.batch_chunk > (uint32_t)kMaxBatchPerLaunch) return fail("batch_chunk above the per-launch limit");
  if (t.row_log2) {
    if ((int)t.log2_len <= lmax) return fail("row_log2 applies to two-pass lengths only");
    if ((int)t.row_log2 > kMaxPassLog || (int)t.log2_len - (int)t.row_log2 < 1 ||
        (int)t.log2_len - (int)t.row_log2 > kMaxPassLog)
      return fail("row_log2 must leave both passes 1..12 stages");
  }
  const Plan base = make_plan((int)t.log2_len, (int)t.word_bits, (int)t.row_log2);
  auto pow2 = [](uint32_t v) { return v && !(v & (v - 1)); };
  // whether g sub-transforms per workgroup fit the pass in the given direction(s)
  auto fits = [&](PassKind kind, int n, uint32_t g, bool fwd, bool inv) {
    bool lds_ok = true;
    if (pass_split(n, (int)t.word_bits).kh != 0) {
      for (const bool inverse : {false, true}) {
        if (!(inverse ? inv : fwd)) continue;
        PassParams pp{};
        pp.kind = kind;
        pp.inverse = inverse;
        pp.word_bits = (int)t.word_bits;
        pp.n = n;
        pp.group = (int)g;
        lds_ok = lds_ok && pass_lds_bytes(pp) != 0;
      }
    }
    return lds_ok && pass_tpt(n, (int)t.word_bits) * (int)g <= kMaxPassThreads;
  };
  if (t.g_cols) {
    if (!base.split || !pow2(t.g_cols) || t.g_cols > (1u << base.c) || !fits(PassKind::kCols, base.r, t.g_cols, true, true))
      return fail("g_cols must be a power of two that fits the column pass");
  }
  if (t.g_rows) {
    if (!base.split || !pow2(t.g_rows) || t.g_rows > (1u << base.r) ||
        !fits(PassKind::kRows, base.c, t.g_rows, true, t.g_rows_inv == 0))
      return fail("g_rows must be a power of two that fits the row pass");
  }
  if (t.g_rows_inv) {
    if (!base.split || !pow2(t.g_rows_inv) || t.g_rows_inv > (1u << base.r) ||
        !fits(PassKind::kRows, base.c, t.g_rows_inv, false, true))
      return fail("g_rows_inv must be a power of two that fits the row pass");
  }
  return HNTT_OK;
}

Plan effective_plan(const hntt_ctx *ctx, int l, int word_bits) {
  auto it = ctx->tuning.find(std::make_pair(l, word_bits));
  Plan pl = make_plan(l, word_bits, it != ctx->tuning.end() ? (int)it->second.row_log2 : 0);
  if (it != ctx->tuning.end()) {
    if (it->second.g_cols) pl.g_cols = (int)it->second.g_cols;
    if (it->second.g_rows) pl.g_rows = (int)it->second.g_rows;
    pl.g_rows_inv = it->second.g_rows_inv ? (int)it->second.g_rows_inv : pl.g_rows;
    if (it->second.batch_chunk) pl.chunk = (int)it->second.batch_chunk;
  }
  return pl;
}

// p^-1 mod 2^bits for odd p (Newton's iteration doubles the correct low bits).
static uint64_t inv_mod_beta(uint64_t p, int bits) {
  uint64_t x = p;  // p p = 1 mod 8
  for (int i = 0; i < 5; ++i) x *= 2 - p * x;
  return bits == 64 ? x : (x & 0xFFFFFFFFull);
}

// Table entries of one twiddle W: (W, floor(W beta / p)) in Shoup form, or the
// single word W beta mod p in Montgomery form.
struct TableForm {
  uint64_t p;
  int bits;
  bool mont;
  uint64_t beta_mod_p;
  TableForm(uint64_t p_, int bits_, bool mont_) : p(p_), bits(bits_), mont(mont_) {
    beta_mod_p = powmod(2 % p_, (uint64_t)bits_, p_);
  }
  size_t words() const { return mont ? 1 : 2; }
  void put(std::vector<uint64_t> &v, size_t idx, uint64_t w) const {
    if (mont) {
      v[idx] = mulmod(w, beta_mod_p, p);
    } else {
      v[2 * idx] = w;
      v[2 * idx + 1] = shoup_constant(w, p, bits);
    }
  }
};

// Per-stage ("heap") table for a transform of length N = 2^n with root w_N:
// entry (1 << b) + k, b < n, k < 2^b, holds W = w_N^(k << (n-1-b)), the twiddle
// of the stage that pairs position bit b, in the table form.  Entry 0 holds 1.
static void heap_table(uint64_t root, int n, const TableForm &form, std::vector<uint64_t> &out) {
  const uint64_t p = form.p;
  const size_t N = (size_t)1 << n;
  std::vector<uint64_t> pw(N / 2 > 0 ? N / 2 : 1);
  uint64_t x = 1;
  for (size_t j = 0; j < pw.size(); ++j) {
    pw[j] = x;
    x = mulmod(x, root, p);
  }
  out.assign(form.words() * N, 0);
  form.put(out, 0, 1);
  for (int b = 0; b < n; ++b)
    for (size_t k = 0; k < ((size_t)1 << b); ++k) form.put(out, ((size_t)1 << b) + k, pw[k << (n - 1 - b)]);
}

// Device copies of one table set, held locally until every upload has succeeded:
// a failure part-way frees what was uploaded and leaves the context's buffers and
// byte count as they were.
struct PendingUploads {
  std::vector<std::unique_ptr<DeviceBuffer>> bufs;
  size_t bytes = 0;
  void commit(hntt_ctx *ctx) {
    for (auto &b : bufs) ctx->buffers.push_back(std::move(b));
    bufs.clear();
    ctx->bytes_held += bytes;
    bytes = 0;
  }
};

int upload(hntt_ctx *ctx, PendingUploads &pend, const std::vector<uint64_t> &src, int bits, const void **out) {
  const size_t bytes = src.size() * (bits / 8);
  if (ctx->budget && ctx->bytes_held + pend.bytes + bytes > ctx->budget)
    return set_error(ctx, HNTT_ENOMEM, "memory budget of %zu bytes exceeded", ctx->budget);
  auto buf = std::make_unique<DeviceBuffer>();
  if (bytes) {
    hipError_t e = hipMalloc(&buf->ptr, bytes);
    if (e != hipSuccess) {
      buf->ptr = nullptr;
      return hip_status(ctx, e, "hipMalloc(twiddle table)");
    }
    buf->bytes = bytes;
    if (bits == 32) {
      std::vector<uint32_t> narrow(src.begin(), src.end());
      e = hipMemcpy(buf->ptr, narrow.data(), bytes, hipMemcpyHostToDevice);
    } else {
      e = hipMemcpy(buf->ptr, src.data(), bytes, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return hip_status(ctx, e, "hipMemcpy(twiddle table)");
  }
  pend.bytes += bytes;
  *out = buf->ptr;
  pend.bufs.push_back(std::move(buf));
  return HNTT_OK;
}

const Tables *find_tables(const hntt_ctx *ctx, uint64_t p, uint64_t omega, int l, int bits, bool mont, int row_log2) {
  auto it = ctx->tables.find(std::make_tuple(p, omega, l, bits, mont, make_plan(l, bits, row_log2).c));
  return it == ctx->tables.end() ? nullptr : &it->second;
}

// Twiddle tables for one (p, omega, l, word_bits, form): built on the host once and kept on the device.
int get_tables(hntt_ctx *ctx, uint64_t p, uint64_t omega, int l, int bits, bool mont, int row_log2,
               const Tables **out) {
  const auto key = std::make_tuple(p, omega, l, bits, mont, make_plan(l, bits, row_log2).c);
  auto it = ctx->tables.find(key);
  if (it != ctx->tables.end()) {
    *out = &it->second;
    return HNTT_OK;
  }
  Tables t{};
  t.plan = make_plan(l, bits, row_log2);
  t.mont = mont;
  const TableForm form(p, bits, mont);
  const uint64_t omega_inv = powmod(omega, p - 2, p);
  const uint64_t L = 1ull << l;
  const uint64_t linv = powmod(L % p, p - 2, p);
  t.linv = mont ? mulmod(linv, form.beta_mod_p, p) : linv;
  t.linv_p = mont ? 0 : shoup_constant(linv, p, bits);
  t.jinv = inv_mod_beta(p, bits);
  std::vector<uint64_t> tab;
  PendingUploads pend;
  int rc;
  auto table = [&](uint64_t root, int n, const void **dst) -> int {
    heap_table(root, n, form, tab);
    return upload(ctx, pend, tab, bits, dst);
  };
  if (!t.plan.split) {
    if ((rc = table(omega, l, &t.fwd))) return rc;
    if ((rc = table(omega_inv, l, &t.inv))) return rc;
  } else {
    const int r = t.plan.r, c = t.plan.c;
    const uint64_t R = 1ull << r, C = 1ull << c;
    // column transforms (length R) use omega^C; row transforms (length C) use omega^R
    if ((rc = table(powmod(omega, C, p), r, &t.fwd))) return rc;
    if ((rc = table(powmod(omega_inv, C, p), r, &t.inv))) return rc;
    if ((rc = table(powmod(omega, R, p), c, &t.row_fwd))) return rc;
    if ((rc = table(powmod(omega_inv, R, p), c, &t.row_inv))) return rc;
    // Split twiddles, one row-major table per direction (see Edge in ntt_pass.hip).
    // Row B (s = rev_r(B)) needs, at row position pos = hi 2^sf + lo, the factor
    // omega^(s pos) (forward, applied as the row pass loads the word) or
    // L^-1 omega^(-s pos) (inverse, applied as the row pass stores it), where
    // sf = c - KH(c) is the boundary of the row pass's high register round.  Each
    // row holds [low factors z^lo | high factors z^(hi 2^sf) (times L^-1 in the
    // inverse) | folded low factors z^lo W(lo)], z = omega^(+-s), W(lo) being the
    // twiddle of the row-transform stage that pairs bit sf at index lo,
    // (omega^(+-R))^(lo 2^(c-1-sf)): the low factor is folded into that stage (Fold
    // in ntt_pass.hip).
    const RoundSplit rs_c = pass_split(c, bits);
    const int sf = c - rs_c.kh;
    const uint64_t Sf = 2 * (1ull << sf) + (1ull << (c - sf));
    std::vector<uint64_t> f(form.words() * R * Sf), iv(form.words() * R * Sf);
    auto put = [&](std::vector<uint64_t> &v, uint64_t idx, uint64_t w) { form.put(v, idx, w); };
    const uint64_t w_row[2] = {powmod(omega, R, p), powmod(omega_inv, R, p)};
    for (int dir = 0; dir < 2; ++dir) {
      std::vector<uint64_t> &dst = dir ? iv : f;
      const uint64_t root = dir ? omega_inv : omega;
      const uint64_t hscale = dir ? linv : 1;
      // twiddle step of the stage pairing bit sf (used only when the row pass has two rounds)
      const uint64_t wstage = sf < c ? powmod(w_row[dir], 1ull << (c - 1 - sf), p) : 1;
      for (uint64_t B = 0; B < R; ++B) {
        const uint64_t ws = powmod(root, bitrev((unsigned)B, r), p);  // z = omega^(+-s)
        const uint64_t wsh = powmod(ws, 1ull << sf, p);                // z^(2^sf)
        const uint64_t fold0 = B * Sf + (1ull << sf) + (1ull << (c - sf));
        uint64_t x = 1, ws_lo = 1;
        for (uint64_t lo = 0; lo < (1ull << sf); ++lo, x = mulmod(x, ws, p), ws_lo = mulmod(ws_lo, wstage, p)) {
          put(dst, B * Sf + lo, x);
          put(dst, fold0 + lo, mulmod(x, ws_lo, p));
        }
        x = hscale;
        for (uint64_t hi = 0; hi < (1ull << (c - sf)); ++hi, x = mulmod(x, wsh, p))
          put(dst, B * Sf + (1ull << sf) + hi, x);
      }
    }
    if ((rc = upload(ctx, pend, f, bits, &t.tt_fwd))) return rc;
    if ((rc = upload(ctx, pend, iv, bits, &t.tt_inv))) return rc;
  }
  pend.commit(ctx);
  auto ins = ctx->tables.emplace(key, t);
  *out = &ins.first->second;
  return HNTT_OK;
}

int ensure_device(hntt_ctx *ctx) {
  if (ctx->device_ready) return HNTT_OK;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0) return set_error(ctx, HNTT_EDEVICE, "no HIP device available");
  if (ctx->device >= count) return set_error(ctx, HNTT_EINVAL, "device %d does not exist", ctx->device);
  ctx->device_ready = true;
  return HNTT_OK;
}

std::string pass_name(const PassParams &pp) {
  const char *kind = pp.kind == PassKind::kWhole ? "whole" : pp.kind == PassKind::kRows ? "rows" : "cols";
  char buf[96];
  const char *pol = pp.policy == kPolicyMont ? "mont" : pp.policy == kPolicyLazy ? "lazy" : "plain";
  const char *dir = pp.fuse_inverse ? "fwdmulinv" : pp.inverse ? "inv" : "fwd";
  snprintf(buf, sizeof buf, "%s_%s_%s_u%d_n%d", kind, dir, pol, pp.word_bits, pp.n);
  return buf;
}

// Run one launch; with tracing on, bracket it with HIP events on the launch stream.
hipError_t trace_launch(hntt_ctx *ctx, const std::string &name, hipStream_t stream,
                        const std::function<hipError_t()> &launch) {
  if (!ctx->trace) return launch();
  TraceEvent ev{name, nullptr, nullptr};
  hipError_t e = hipEventCreate(&ev.start);
  if (e != hipSuccess) return e;
  if ((e = hipEventCreate(&ev.stop)) != hipSuccess) {
    (void)hipEventDestroy(ev.start);
    return e;
  }
  (void)hipEventRecord(ev.start, stream);
  e = launch();
  (void)hipEventRecord(ev.stop, stream);
  ctx->trace_pending.push_back(ev);
  return e;
}

hipError_t launch_traced(hntt_ctx *ctx, const PassParams &pp, const BatchPtrs &bp, hipStream_t stream) {
  return trace_launch(ctx, pass_name(pp), stream, [&]() { return launch_pass(pp, bp, stream); });
}

// Run every pass of one transform direction over a batch sharing (p, omega, l, word_bits).
int run_transform(hntt_ctx *ctx, const Tables &t, const Plan &plan, const std::vector<void *> &ptrs, uint64_t p,
                  int l, int bits, bool inverse, uint32_t flags, hipStream_t stream) {
  const int policy = (flags & HNTT_PLAIN) ? kPolicyPlain : (flags & HNTT_MONT) ? kPolicyMont : kPolicyLazy;
  const bool norm = !(flags & HNTT_NO_NORMALIZE);
  const size_t chunk = (size_t)std::max(1, std::min(plan.chunk, kMaxBatchPerLaunch));
  for (size_t off = 0; off < ptrs.size(); off += chunk) {
    BatchPtrs bp{};
    const int nb = (int)std::min<size_t>(chunk, ptrs.size() - off);
    for (int i = 0; i < nb; ++i) bp.ptr[i] = reinterpret_cast<uint64_t>(ptrs[off + i]);
    PassParams pp{};
    pp.word_bits = bits;
    pp.policy = policy;
    pp.inverse = inverse;
    pp.nbatch = nb;
    pp.p = p;
    pp.jinv = t.jinv;
    hipError_t e;
    if (!plan.split) {
      pp.kind = PassKind::kWhole;
      pp.n = l;
      pp.log_other = 0;
      pp.group = 1;
      pp.normalize = norm;
      pp.tw = inverse ? t.inv : t.fwd;
      pp.scale_w = t.linv;
      pp.scale_wp = t.linv_p;
      if ((e = launch_traced(ctx, pp, bp, stream)) != hipSuccess) return hip_status(ctx, e, "launch(whole)");
      continue;
    }
    PassParams cols = pp, rows = pp;
    cols.kind = PassKind::kCols;
    cols.n = plan.r;
    cols.log_other = plan.c;
    cols.group = plan.g_cols;
    cols.tw = inverse ? t.inv : t.fwd;
    cols.tt = nullptr;  // the split twiddle belongs to the row pass (both directions)
    rows.kind = PassKind::kRows;
    rows.n = plan.c;
    rows.log_other = plan.r;
    rows.group = inverse ? plan.g_rows_inv : plan.g_rows;
    rows.tw = inverse ? t.row_inv : t.row_fwd;
    rows.tt = inverse ? t.tt_inv : t.tt_fwd;
    if (!inverse) {
      cols.normalize = false;
      rows.normalize = norm;
      if ((e = launch_traced(ctx, cols, bp, stream)) != hipSuccess) return hip_status(ctx, e, "launch(cols)");
      if ((e = launch_traced(ctx, rows, bp, stream)) != hipSuccess) return hip_status(ctx, e, "launch(rows)");
    } else {
      rows.normalize = false;
      cols.normalize = norm;
      if ((e = launch_traced(ctx, rows, bp, stream)) != hipSuccess) return hip_status(ctx, e, "launch(rows)");
      if ((e = launch_traced(ctx, cols, bp, stream)) != hipSuccess) return hip_status(ctx, e, "launch(cols)");
    }
  }
  return HNTT_OK;
}

// HNTT_VALIDATE: one range check per array, all lowering one device word to the
// smallest index with a word >= its bound, then a wait for the stream to read it.
// `arrays` holds (data, words, word_bits, bound, index).
struct CheckedArray {
  const void *data;
  uint64_t len;
  int word_bits;
  uint64_t bound;
  uint32_t index;
};

int check_inputs(hntt_ctx *ctx, const std::vector<CheckedArray> &arrays, hipStream_t stream) {
  if (!ctx->check_flag) {
    hipError_t e = hipMalloc(&ctx->check_flag, 256);
    if (e != hipSuccess) {
      ctx->check_flag = nullptr;
      return hip_status(ctx, e, "hipMalloc(check flag)");
    }
  }
  const uint32_t none = 0xffffffffu;
  hipError_t e = launch_set_flag(ctx->check_flag, none, stream);
  for (size_t i = 0; e == hipSuccess && i < arrays.size(); ++i) {
    const CheckedArray &a = arrays[i];
    e = launch_range_check(a.word_bits, a.data, a.len, a.bound, a.index, ctx->check_flag, stream);
  }
  uint32_t first = none;
  if (e == hipSuccess) e = hipMemcpyAsync(&first, ctx->check_flag, sizeof first, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_status(ctx, e, "input check");
  if (first != none) return set_error(ctx, HNTT_EINVAL, "descriptor %u: an input word is not below p", first);
  return HNTT_OK;
}

int transform(hntt_ctx *ctx, const hntt_desc *descs, size_t n, uint32_t flags, void *stream, bool inverse) {
  if (!ctx) return HNTT_EINVAL;
  ctx->last_error.clear();
  if (n && !descs) return set_error(ctx, HNTT_EINVAL, "descs is NULL");
  if (flags & ~(HNTT_PLAIN | HNTT_NO_NORMALIZE | HNTT_MONT | HNTT_VALIDATE))
    return set_error(ctx, HNTT_EINVAL, "unknown flag bits");
  if ((flags & HNTT_PLAIN) && (flags & HNTT_MONT))
    return set_error(ctx, HNTT_EINVAL, "HNTT_PLAIN and HNTT_MONT select different butterflies");
  // group descriptors that share parameters; validate everything before enqueueing anything
  std::map<std::tuple<uint64_t, uint64_t, int, int>, std::vector<void *>> groups;
  for (size_t i = 0; i < n; ++i) {
    int rc = check_desc(ctx, descs[i], flags);
    if (rc) return rc;
    groups[std::make_tuple(descs[i].p, descs[i].omega, (int)descs[i].log2_len, (int)descs[i].word_bits)].push_back(
        descs[i].data);
  }
  if (n == 0) return HNTT_OK;
  int rc = ensure_device(ctx);
  if (rc) return rc;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return set_error(ctx, HNTT_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
  if (flags & HNTT_VALIDATE) {
    std::vector<CheckedArray> arrays;
    for (size_t i = 0; i < n; ++i)
      arrays.push_back({descs[i].data, (uint64_t)1 << descs[i].log2_len, (int)descs[i].word_bits, descs[i].p,
                        (uint32_t)i});
    if ((rc = check_inputs(ctx, arrays, (hipStream_t)stream))) return rc;
  }
  for (auto &kv : groups) {
    const uint64_t p = std::get<0>(kv.first), omega = std::get<1>(kv.first);
    const int l = std::get<2>(kv.first), bits = std::get<3>(kv.first);
    const Tables *t = nullptr;
    if ((rc = get_tables(ctx, p, omega, l, bits, (flags & HNTT_MONT) != 0, effective_plan(ctx, l, bits).c, &t)))
      return rc;
    const Plan plan = effective_plan(ctx, l, bits);
    if ((rc = run_transform(ctx, *t, plan, kv.second, p, l, bits, inverse, flags, (hipStream_t)stream))) return rc;
  }
  return HNTT_OK;
}

}  // namespace hntt

// ==================================================================================================
extern "C" {

int hntt_create(hntt_ctx **out, int device, size_t mem_budget_bytes) {
  if (!out || device < 0) return HNTT_EINVAL;
  hntt_ctx *c = new (std::nothrow) hntt_ctx();
  if (!c) return HNTT_ENOMEM;
  c->device = device;
  c->budget = mem_budget_bytes;
  *out = c;
  return HNTT_OK;
}

void hntt_destroy(hntt_ctx *ctx) {
  if (!ctx) return;
  if (ctx->device_ready) {
    DeviceGuard guard(ctx->device);
    ctx->release_poly_cache();
    ctx->release_device_state();
    ctx->buffers.clear();
  }
  delete ctx;
}

const char *hntt_strerror(int status) {
  switch (status) {
    case HNTT_OK: return "success";
    case HNTT_EINVAL: return "invalid argument";
    case HNTT_EUNSUPPORTED: return "unsupported parameters";
    case HNTT_ENOMEM: return "out of device memory or over the context budget";
    case HNTT_EDEVICE: return "HIP device error";
    case HNTT_EBUSY: return "busy: request not admitted";
    default: return "unknown status";
  }
}

const char *hntt_last_error(const hntt_ctx *ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int hntt_ntt_forward(hntt_ctx *ctx, const hntt_desc *descs, size_t n, uint32_t flags, void *stream) {
  return transform(ctx, descs, n, flags, stream, false);
}

int hntt_ntt_inverse(hntt_ctx *ctx, const hntt_desc *descs, size_t n, uint32_t flags, void *stream) {
  return transform(ctx, descs, n, flags, stream, true);
}

int hntt_validate(hntt_ctx *ctx, const hntt_desc *descs, size_t n, uint32_t flags) {
  if (!ctx) return HNTT_EINVAL;
  ctx->last_error.clear();
  if (n && !descs) return set_error(ctx, HNTT_EINVAL, "descs is NULL");
  if (flags & ~(HNTT_PLAIN | HNTT_NO_NORMALIZE | HNTT_MONT | HNTT_VALIDATE))
    return set_error(ctx, HNTT_EINVAL, "unknown flag bits");
  if ((flags & HNTT_PLAIN) && (flags & HNTT_MONT))
    return set_error(ctx, HNTT_EINVAL, "HNTT_PLAIN and HNTT_MONT select different butterflies");
  for (size_t i = 0; i < n; ++i) {
    int rc = check_desc(ctx, descs[i], flags);
    if (rc) return rc;
  }
  return HNTT_OK;
}

int hntt_pointwise_mul(hntt_ctx *ctx, const hntt_pw_desc *descs, size_t n, uint32_t flags, void *stream) {
  if (!ctx) return HNTT_EINVAL;
  ctx->last_error.clear();
  if (n && !descs) return set_error(ctx, HNTT_EINVAL, "descs is NULL");
  if (flags & ~HNTT_VALIDATE) return set_error(ctx, HNTT_EINVAL, "pointwise_mul takes only HNTT_VALIDATE");
  for (size_t i = 0; i < n; ++i) {
    const hntt_pw_desc &d = descs[i];
    if (d.word_bits != 32 && d.word_bits != 64) return set_error(ctx, HNTT_EINVAL, "word_bits must be 32 or 64");
    if (d.reserved) return set_error(ctx, HNTT_EINVAL, "reserved field must be 0");
    if (d.len && (!d.a || !d.b || !d.c)) return set_error(ctx, HNTT_EINVAL, "NULL operand");
    if (d.p < 3 || !(d.p & 1)) return set_error(ctx, HNTT_EINVAL, "p must be odd and >= 3");
    if (d.p >= (1ull << (d.word_bits - 2)))
      return set_error(ctx, HNTT_EUNSUPPORTED, "pointwise_mul needs p < 2^%u", d.word_bits - 2);
  }
  if (n == 0) return HNTT_OK;
  int rc = ensure_device(ctx);
  if (rc) return rc;
  DeviceGuard guard(ctx->device);
  if (!guard.ok) return set_error(ctx, HNTT_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
  if (flags & HNTT_VALIDATE) {
    std::vector<CheckedArray> arrays;
    for (size_t i = 0; i < n; ++i) {
      const hntt_pw_desc &d = descs[i];
      arrays.push_back({d.a, d.len, (int)d.word_bits, d.p, (uint32_t)i});
      arrays.push_back({d.b, d.len, (int)d.word_bits, d.p, (uint32_t)i});
    }
    if ((rc = check_inputs(ctx, arrays, (hipStream_t)stream))) return rc;
  }
  for (size_t i = 0; i < n; ++i) {
    const hntt_pw_desc &d = descs[i];
    hipError_t e = launch_pointwise((int)d.word_bits, d.p, d.a, d.b, d.c, d.len, (hipStream_t)stream);
    if (e != hipSuccess) return hip_status(ctx, e, "launch(pointwise)");
  }
  return HNTT_OK;
}

int hntt_set_tuning(hntt_ctx *ctx, const hntt_tuning *t) {
  if (!ctx || !t) return HNTT_EINVAL;
  ctx->last_error.clear();
  std::string why;
  if (check_tuning(*t, &why)) return set_error(ctx, HNTT_EINVAL, "%s", why.c_str());
  ctx->tuning[std::make_pair((int)t->log2_len, (int)t->word_bits)] = *t;
  return HNTT_OK;
}

int hntt_get_plan(hntt_ctx *ctx, uint32_t log2_len, uint32_t word_bits, hntt_tuning *out) {
  if (!ctx || !out || (word_bits != 32 && word_bits != 64)) return HNTT_EINVAL;
  const int lmax = max_whole_log((int)word_bits);
  if (log2_len < 1 || (int)log2_len > 2 * lmax) return set_error(ctx, HNTT_EUNSUPPORTED, "no plan for this length");
  const Plan pl = effective_plan(ctx, (int)log2_len, (int)word_bits);
  out->log2_len = log2_len;
  out->word_bits = word_bits;
  out->g_cols = pl.split ? (uint32_t)pl.g_cols : 0;
  out->g_rows = pl.split ? (uint32_t)pl.g_rows : 0;
  out->batch_chunk = (uint32_t)pl.chunk;
  out->row_log2 = (uint32_t)pl.c;
  out->g_rows_inv = pl.split ? (uint32_t)pl.g_rows_inv : 0;
  return HNTT_OK;
}

int hntt_trace_enable(hntt_ctx *ctx, int enable) {
  if (!ctx) return HNTT_EINVAL;
  ctx->trace = enable != 0;
  return HNTT_OK;
}

int hntt_trace_reset(hntt_ctx *ctx) {
  if (!ctx) return HNTT_EINVAL;
  for (auto &ev : ctx->trace_pending) {
    (void)hipEventSynchronize(ev.stop);
    (void)hipEventDestroy(ev.start);
    (void)hipEventDestroy(ev.stop);
  }
  ctx->trace_pending.clear();
  ctx->trace_acc.clear();
  return HNTT_OK;
}

int hntt_trace_read(hntt_ctx *ctx, char *buf, size_t *len) {
  if (!ctx || !len) return HNTT_EINVAL;
  int status = HNTT_OK;
  for (auto &ev : ctx->trace_pending) {
    float ms = 0;
    if (hipEventSynchronize(ev.stop) != hipSuccess || hipEventElapsedTime(&ms, ev.start, ev.stop) != hipSuccess)
      status = set_error(ctx, HNTT_EDEVICE, "trace event failed");
    TraceAcc &a = ctx->trace_acc[ev.name];
    a.launches += 1;
    a.total_ms += ms;
    (void)hipEventDestroy(ev.start);
    (void)hipEventDestroy(ev.stop);
  }
  ctx->trace_pending.clear();
  std::string json = "{";
  bool first = true;
  for (auto &kv : ctx->trace_acc) {
    char item[256];
    snprintf(item, sizeof item, "%s\"%s\": {\"launches\": %llu, \"total_ms\": %.6f}", first ? "" : ", ",
             kv.first.c_str(), (unsigned long long)kv.second.launches, kv.second.total_ms);
    json += item;
    first = false;
  }
  json += "}";
  const size_t need = json.size() + 1;
  if (!buf || *len < need) {
    *len = need;
    return status ? status : HNTT_ENOMEM;
  }
  memcpy(buf, json.c_str(), need);
  *len = need;
  return status;
}

int hntt_is_prime(uint64_t n) { return is_prime_u64(n) ? 1 : 0; }

uint64_t hntt_primitive_root(uint64_t p) { return primitive_root(p); }

int hntt_root_of_unity(uint64_t p, uint32_t log2_len, uint64_t *omega_out) {
  if (!omega_out || log2_len > 63) return HNTT_EINVAL;
  const uint64_t g = primitive_root(p);
  if (!g) return HNTT_EINVAL;
  if ((p - 1) % (1ull << log2_len)) return HNTT_EINVAL;
  *omega_out = powmod(g, (p - 1) >> log2_len, p);
  return HNTT_OK;
}

uint64_t hntt_find_prime(uint32_t bits, uint32_t v) { return find_prime(bits, v); }

int hntt_shoup_constant(uint64_t w, uint64_t p, uint32_t word_bits, uint64_t *wprime_out) {
  if (!wprime_out || (word_bits != 32 && word_bits != 64) || p < 2 || w >= p) return HNTT_EINVAL;
  if (word_bits == 32 && p > 0xFFFFFFFFull) return HNTT_EINVAL;
  *wprime_out = shoup_constant(w, p, (int)word_bits);
  return HNTT_OK;
}

int hntt_debug_butterfly(hntt_ctx *ctx, int kind, uint32_t word_bits, uint64_t p, const void *x, const void *y,
                         const void *w, const void *wprime, void *xo, void *yo, size_t n, void *stream) {
  if (!ctx) return HNTT_EINVAL;
  ctx->last_error.clear();
  if (kind < 0 || kind > 5) return set_error(ctx, HNTT_EINVAL, "kind must be 0..5");
  if (word_bits != 32 && word_bits != 64) return set_error(ctx, HNTT_EINVAL, "word_bits must be 32 or 64");
  if (n && (!x || !y || !w || !wprime || !xo || !yo)) return set_error(ctx, HNTT_EINVAL, "NULL array");
  const unsigned limit_bits = word_bits - ((kind == 0 || kind == 3) ? 1 : 2);
  if (p < 3 || (limit_bits < 64 && p >= (1ull << limit_bits)))
    return set_error(ctx, HNTT_EUNSUPPORTED, "p out of range for this butterfly");
  if (n == 0) return HNTT_OK;
  int rc = ensure_device(ctx);
  if (rc) return rc;
  DeviceGuard guard(ctx->device);
  hipError_t e = launch_debug_butterfly(kind, (int)word_bits, p, x, y, w, wprime, xo, yo, n, (hipStream_t)stream);
  return hip_status(ctx, e, "launch(debug_butterfly)");
}

}  // extern "C"
