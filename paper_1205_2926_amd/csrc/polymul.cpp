// Exact polynomial products through three NTT primes and Chinese remaindering
// (the application named in Section 1 of the paper): host planning, device
// metadata, and the capture-safe enqueue that is recorded once into a HIP graph
// and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "hntt.h"
#include "hntt_internal.hpp"
#include "ntt_kernels.hpp"
#include "numtheory.hpp"
#include "polymul_kernels.hpp"
#include "static_scratch.hpp"

using namespace hntt;

namespace {

constexpr uint64_t kPrimes[3] = {998244353ull, 754974721ull, 167772161ull};
constexpr int kMaxPolyLog = 23;  // 2^23 divides q - 1 for all three primes
constexpr int kChunkWords = 1024;

int perr(hntt_ctx *ctx, int status, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int perr(hntt_ctx *ctx, int status, const char *fmt, ...) {
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

int hip_err(hntt_ctx *ctx, hipError_t e, const char *what) {
  if (e == hipSuccess) return HNTT_OK;
  return perr(ctx, e == hipErrorOutOfMemory ? HNTT_ENOMEM : HNTT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

uint32_t shoup32(uint64_t w, uint64_t q) { return (uint32_t)shoup_constant(w, q, 32); }

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int log2_padded(uint32_t na, uint32_t nb) {
  const uint32_t m = std::max(na, nb);
  int l = 0;
  while ((1u << l) < m) ++l;
  return l + 1;  // L = 2 * nextpow2(max(na, nb))
}

// Sizes and arena layout of a batch (host only).
struct Sizing {
  std::vector<int> logs;
  std::vector<int> class_count;
  size_t ws_words = 0, chunks_ws = 0, chunks_out = 0;
  size_t off_pairs = 0, off_cws = 0, off_cout = 0, off_xf = 0, off_state = 0, off_carry = 0, total = 0;
};

// `big`: products of base-2^32 limb integers (na + nb uint32 limbs out) instead of
// uint64 coefficient vectors (na + nb - 1 coefficients out).
int size_batch(hntt_ctx *ctx, const hntt_poly_desc *descs, size_t n, bool check_ptrs, Sizing *sz, bool big = false) {
  sz->logs.assign(n, 0);
  sz->class_count.assign(kMaxPolyLog + 1, 0);
  for (size_t i = 0; i < n; ++i) {
    const hntt_poly_desc &d = descs[i];
    if (d.na == 0 || d.nb == 0) return perr(ctx, HNTT_EINVAL, "product %zu: empty operand", i);
    if (check_ptrs) {
      if (!d.a || !d.b || !d.out) return perr(ctx, HNTT_EINVAL, "product %zu: NULL pointer", i);
      if ((reinterpret_cast<uintptr_t>(d.a) | reinterpret_cast<uintptr_t>(d.b)) % 4 ||
          reinterpret_cast<uintptr_t>(d.out) % (big ? 4 : 8))
        return perr(ctx, HNTT_EINVAL, "product %zu: misaligned pointer", i);
    }
    const int l = log2_padded(d.na, d.nb);
    if (l > kMaxPolyLog)
      return perr(ctx, HNTT_EUNSUPPORTED, "product %zu: padded length 2^%d above 2^%d", i, l, kMaxPolyLog);
    sz->logs[i] = l;
    sz->ws_words += 6ull << l;
    sz->chunks_ws += ((1ull << l) / 2 + kChunkWords - 1) / kChunkWords;  // preparation covers the lower half
    sz->chunks_out += ((uint64_t)d.na + d.nb - (big ? 0 : 1) + kChunkWords - 1) / kChunkWords;
    sz->class_count[l]++;
  }
  if (sz->chunks_ws > (1u << 30) || sz->chunks_out > (1u << 30))
    return perr(ctx, HNTT_EUNSUPPORTED, "batch too large");
  size_t n_xf = 0;
  for (int l = 0; l <= kMaxPolyLog; ++l) n_xf += (size_t)sz->class_count[l] * 9;
  sz->off_pairs = align_up(sz->ws_words * 4, 256);
  sz->off_cws = align_up(sz->off_pairs + n * sizeof(PolyPair), 256);
  sz->off_cout = align_up(sz->off_cws + sz->chunks_ws * sizeof(ChunkEntry), 256);
  sz->off_xf = align_up(sz->off_cout + sz->chunks_out * sizeof(ChunkEntry), 256);
  // large-integer mode: carry state and carry-in of every output chunk
  sz->off_state = align_up(sz->off_xf + n_xf * sizeof(XformEntry), 256);
  sz->off_carry = align_up(sz->off_state + (big ? sz->chunks_out * 4 : 0), 256);
  sz->total = align_up(sz->off_carry + (big ? sz->chunks_out * 4 : 0), 256);
  return HNTT_OK;
}

struct ClassWork {
  int l;
  int ws0, ws1, out0, out1;  // the class's range of preparation and output chunks
  Plan plan;  // the class's split and schedule, fixed when the plan is made
  int nfwd, ninv;               // nfwd: entries of each forward table
  const XformEntry *fwd_a, *fwd_b, *inv;  // device tables inside the arena
  const Tables *tab[3];
};

}  // namespace

struct hntt_polymul_plan {
  hntt_ctx *ctx = nullptr;
  uint32_t flags = 0;
  bool big = false;  // large-integer products (limbs out) instead of coefficient vectors
  size_t n = 0;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  bool owns_arena = false;
  PolyArgs args{};
  std::vector<ClassWork> classes;
  std::vector<unsigned char> host_meta;  // kept alive until the plan is destroyed
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool graph_failed = false;
  std::string graph_error;  // why recording the graph failed
  int exec_mode = HNTT_EXEC_NONE;
  std::vector<hntt_poly_desc> descs;  // for the one-shot cache
};

namespace hntt {

// B_k's last forward pass multiplies into A_k and runs A_k's first inverse pass on
// the product in the same launch (PassParams::fuse_inverse), saving the product's
// round trip through memory; when false the product is written and the inverse
// starts with its own launch.
constexpr bool kFuseProductInverse = true;

// Enqueue the transforms of a length class listed in a device table.  `which`:
// 0 = forward of the A_k, 1 = forward of the B_k with the pointwise product fused
// into their last pass (it multiplies into A_k, which starts L words earlier) and,
// with kFuseProductInverse, A_k's first inverse pass after it, 2 = (the rest of) the
// inverse of the A_k.
static int run_class(hntt_ctx *ctx, const ClassWork &cw, int which, uint32_t flags, hipStream_t s) {
  const Plan &plan = cw.plan;
  const bool inverse = which == 2;
  const XformEntry *table = which == 0 ? cw.fwd_a : which == 1 ? cw.fwd_b : cw.inv;
  const int count = inverse ? cw.ninv : cw.nfwd;
  const uint32_t pm_off = which == 1 ? (1u << cw.l) : 0u;
  const bool fuse = which == 1 && kFuseProductInverse;
  if (count == 0) return HNTT_OK;
  PassParams base{};
  base.word_bits = 32;
  base.policy = (flags & HNTT_PLAIN) ? kPolicyPlain : kPolicyLazy;
  base.inverse = inverse;
  base.nbatch = count;
  base.table = table;
  base.nslots = 3;
  auto slots_for = [&](PassParams &pp, int which) {
    for (int k = 0; k < 3; ++k) {
      const Tables &t = *cw.tab[k];
      SlotParams &sp = pp.slots[k];
      sp.p = kPrimes[k];
      sp.scale_w = t.linv;
      sp.scale_wp = t.linv_p;
      sp.jinv = t.jinv;
      sp.tt = nullptr;
      sp.tw2 = sp.tt2 = nullptr;
      // the split twiddle belongs to the row pass (both directions)
      if (which == 0) {                                               // whole
        sp.tw = inverse ? t.inv : t.fwd;
        if (fuse) sp.tw2 = t.inv;
      } else if (which == 1) {                                        // columns
        sp.tw = inverse ? t.inv : t.fwd;
        sp.tt = nullptr;
      } else {                                                        // rows
        sp.tw = inverse ? t.row_inv : t.row_fwd;
        sp.tt = inverse ? t.tt_inv : t.tt_fwd;
        if (fuse) {
          sp.tw2 = t.row_inv;
          sp.tt2 = t.tt_inv;
        }
      }
    }
  };
  hipError_t e;
  if (!plan.split) {
    if (inverse && kFuseProductInverse) return HNTT_OK;  // done by the fused forward pass of the B_k
    PassParams pp = base;
    pp.kind = PassKind::kWhole;
    pp.n = cw.l;
    pp.log_other = 0;
    pp.group = 1;
    pp.normalize = true;
    pp.pm_off = pm_off;
    pp.fuse_inverse = fuse;
    pp.zero_upper = !inverse;  // padded operands: the upper half is zero
    slots_for(pp, 0);
    if ((e = launch_traced(ctx, pp, BatchPtrs{}, s)) != hipSuccess) return hip_err(ctx, e, "launch(poly whole)");
    return HNTT_OK;
  }
  PassParams cols = base, rows = base;
  cols.kind = PassKind::kCols;
  cols.n = plan.r;
  cols.log_other = plan.c;
  cols.group = plan.g_cols;
  slots_for(cols, 1);
  rows.kind = PassKind::kRows;
  rows.n = plan.c;
  rows.log_other = plan.r;
  rows.group = plan.g_rows;
  slots_for(rows, 2);
  cols.normalize = inverse;
  rows.normalize = !inverse && !fuse;  // the fused inverse row output feeds the inverse column pass
  rows.pm_off = pm_off;
  rows.fuse_inverse = fuse;
  cols.zero_upper = !inverse;  // padded operands: rows in the upper half are zero
  if (!inverse) {
    if ((e = launch_traced(ctx, cols, BatchPtrs{}, s)) != hipSuccess) return hip_err(ctx, e, "launch(poly cols)");
    if ((e = launch_traced(ctx, rows, BatchPtrs{}, s)) != hipSuccess) return hip_err(ctx, e, "launch(poly rows)");
  } else {
    if (!kFuseProductInverse)
      if ((e = launch_traced(ctx, rows, BatchPtrs{}, s)) != hipSuccess) return hip_err(ctx, e, "launch(poly rows)");
    if ((e = launch_traced(ctx, cols, BatchPtrs{}, s)) != hipSuccess) return hip_err(ctx, e, "launch(poly cols)");
  }
  return HNTT_OK;
}

// Parallel branches of a recorded plan (one per length class, up to this many).
constexpr int kGraphBranches = 4;

// Length classes are independent from the preparation to the CRT.  With `branch`
// streams (and one fork event and one join event per stream) class i runs on
// branch[i % nbranch], forked from and joined back into s: recorded into a graph,
// the classes become parallel branches, so that the short launches of the small
// classes need not wait for the long ones of the large classes.
struct Branches {
  hipStream_t *stream = nullptr;
  hipEvent_t *fork = nullptr, *join = nullptr;
  int n = 0;
};

static int enqueue_plan(hntt_polymul_plan *pl, hipStream_t s, const Branches &br = Branches{}) {
  hntt_ctx *ctx = pl->ctx;
  const PolyArgs &a = pl->args;
  hipError_t e;
  int rc;
  const int nb = br.n > 0 ? std::min<int>(br.n, (int)pl->classes.size()) : 0;
  // on branches, coefficient products prepare and recombine each class on its own
  // branch (the preparation and CRT of one class overlap the transforms of others)
  const bool per_class = nb > 0 && !pl->big;
  const auto class_args = [&](const ClassWork &cw) {
    PolyArgs ca = a;
    ca.chunks_ws = a.chunks_ws + cw.ws0;
    ca.nchunks_ws = cw.ws1 - cw.ws0;
    ca.chunks_out = a.chunks_out + cw.out0;
    ca.nchunks_out = cw.out1 - cw.out0;
    return ca;
  };
  if (!per_class &&
      (e = trace_launch(ctx, "poly_prep", s, [&]() { return launch_poly_prep(a, s); })) != hipSuccess)
    return hip_err(ctx, e, "launch(poly prep)");
  for (int b = 0; b < nb; ++b) {
    if ((e = hipEventRecord(br.fork[b], s)) != hipSuccess) return hip_err(ctx, e, "hipEventRecord(fork)");
    if ((e = hipStreamWaitEvent(br.stream[b], br.fork[b], 0)) != hipSuccess)
      return hip_err(ctx, e, "hipStreamWaitEvent(fork)");
  }
  if (nb) {
    // largest classes first, each to the branch with the least work so far (work of a
    // class ~ transforms x L log L); on its branch a class runs its three phases in turn
    std::vector<size_t> order(pl->classes.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    const auto work = [&](size_t i) {
      const ClassWork &cw = pl->classes[i];
      return (double)cw.nfwd * (double)(1ull << cw.l) * cw.l;
    };
    std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return work(x) > work(y); });
    std::vector<double> load(nb, 0.0);
    for (size_t i : order) {
      const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[b] += work(i);
      const hipStream_t st = br.stream[b];
      const PolyArgs ca = class_args(pl->classes[i]);
      if (per_class &&
          (e = trace_launch(ctx, "poly_prep", st, [&]() { return launch_poly_prep(ca, st); })) != hipSuccess)
        return hip_err(ctx, e, "launch(poly prep)");
      for (int which = 0; which < 3; ++which)
        if ((rc = run_class(ctx, pl->classes[i], which, pl->flags, st))) return rc;
      if (per_class &&
          (e = trace_launch(ctx, "poly_crt", st, [&]() { return launch_poly_crt(ca, st); })) != hipSuccess)
        return hip_err(ctx, e, "launch(poly crt)");
    }
  } else {
    for (const ClassWork &cw : pl->classes)
      if ((rc = run_class(ctx, cw, 0, pl->flags, s))) return rc;
    for (const ClassWork &cw : pl->classes)  // B_k transforms; their last pass multiplies into A_k
      if ((rc = run_class(ctx, cw, 1, pl->flags, s))) return rc;
    for (const ClassWork &cw : pl->classes)
      if ((rc = run_class(ctx, cw, 2, pl->flags, s))) return rc;
  }
  for (int b = 0; b < nb; ++b) {
    if ((e = hipEventRecord(br.join[b], br.stream[b])) != hipSuccess) return hip_err(ctx, e, "hipEventRecord(join)");
    if ((e = hipStreamWaitEvent(s, br.join[b], 0)) != hipSuccess) return hip_err(ctx, e, "hipStreamWaitEvent(join)");
  }
  if (pl->big) {
    if ((e = trace_launch(ctx, "big_crt", s, [&]() { return launch_big_crt(a, s); })) != hipSuccess)
      return hip_err(ctx, e, "launch(big crt)");
    if ((e = trace_launch(ctx, "big_carry", s, [&]() { return launch_big_carry(a, s); })) != hipSuccess)
      return hip_err(ctx, e, "launch(big carry)");
  } else if (!per_class &&
             (e = trace_launch(ctx, "poly_crt", s, [&]() { return launch_poly_crt(a, s); })) != hipSuccess) {
    return hip_err(ctx, e, "launch(poly crt)");
  }
  return HNTT_OK;
}

}  // namespace hntt

// Plan a batch of products: coefficient vectors (big = false) or large-integer
// limb products (big = true); descriptors are checked on the host first.
// no_alloc: the workspace is the static device array (given as `workspace`), the
// twiddle tables must already be resident, and nothing is allocated on the device.
static int plan_create(hntt_ctx *ctx, const hntt_poly_desc *descs, size_t n, uint32_t flags, bool big,
                       void *workspace, size_t workspace_bytes, void *stream, hntt_polymul_plan **out,
                       bool no_alloc = false) {
  if (!ctx || !out) return HNTT_EINVAL;
  ctx->last_error.clear();
  *out = nullptr;
  if (n && !descs) return perr(ctx, HNTT_EINVAL, "descs is NULL");
  if (flags & ~(HNTT_PLAIN | HNTT_NO_GRAPH)) return perr(ctx, HNTT_EINVAL, "unknown flag bits");
  if (n > (1u << 24)) return perr(ctx, HNTT_EUNSUPPORTED, "too many products in one plan");
  // host checks first: nothing touches the device before every descriptor is valid
  Sizing sz;
  int rc = size_batch(ctx, descs, n, true, &sz, big);
  if (rc) return rc;
  const std::vector<int> &logs = sz.logs;
  const std::vector<int> &class_count = sz.class_count;
  const size_t chunks_ws = sz.chunks_ws, chunks_out = sz.chunks_out;
  rc = ensure_device(ctx);
  if (rc) return rc;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(ctx->device) != hipSuccess) return perr(ctx, HNTT_EDEVICE, "hipSetDevice failed");
  struct Restore {
    int d;
    ~Restore() {
      if (d >= 0) (void)hipSetDevice(d);
    }
  } restore{prev};

  std::unique_ptr<hntt_polymul_plan> pl(new hntt_polymul_plan());
  pl->ctx = ctx;
  pl->flags = flags;
  pl->big = big;
  pl->n = n;
  pl->descs.assign(descs, descs + n);

  // twiddle tables of every (prime, length) that occurs; built on the host, cached on the context
  std::vector<ClassWork> classes;
  for (int l = 1; l <= kMaxPolyLog; ++l) {
    if (!class_count[l]) continue;
    ClassWork cw{};
    cw.l = l;
    cw.plan = effective_plan(ctx, l, 32);  // the tables below are built for its split
    for (int k = 0; k < 3; ++k) {
      const uint64_t q = kPrimes[k];
      const uint64_t omega = powmod(primitive_root(q), (q - 1) >> l, q);
      if (!no_alloc) {
        if ((rc = get_tables(ctx, q, omega, l, 32, false, cw.plan.c, &cw.tab[k]))) return rc;
      } else if (!(cw.tab[k] = find_tables(ctx, q, omega, l, 32, false, cw.plan.c))) {
        return perr(ctx, HNTT_EUNSUPPORTED,
                    "twiddle tables of padded length 2^%d are not resident on this context (an earlier "
                    "hntt_polymul_crt or plan with products of that length builds them)", l);
      }
    }
    classes.push_back(cw);
  }

  // arena: workspace, then the metadata tables
  const size_t off_pairs = sz.off_pairs, off_cws = sz.off_cws, off_cout = sz.off_cout, off_xf = sz.off_xf;
  const size_t total = sz.total;
  if (no_alloc && !workspace) return perr(ctx, HNTT_EINVAL, "no workspace");
  if (workspace) {
    if (workspace_bytes < total)
      return perr(ctx, HNTT_ENOMEM, "workspace of %zu bytes is smaller than the %zu this plan needs", workspace_bytes,
                  total);
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return perr(ctx, HNTT_EINVAL, "workspace not 256-byte aligned");
    pl->arena = static_cast<char *>(workspace);
    pl->owns_arena = false;
  } else {
    if (ctx->budget && ctx->bytes_held + total > ctx->budget)
      return perr(ctx, HNTT_ENOMEM, "memory budget of %zu bytes exceeded (plan needs %zu)", ctx->budget, total);
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, total);
    if (e != hipSuccess) return hip_err(ctx, e, "hipMalloc(polymul workspace)");
    pl->arena = static_cast<char *>(p);
    pl->owns_arena = true;
    ctx->bytes_held += total;
  }
  pl->arena_bytes = total;

  // host images of the metadata
  std::vector<unsigned char> &meta = pl->host_meta;
  meta.assign(total - off_pairs, 0);
  PolyPair *hp = reinterpret_cast<PolyPair *>(meta.data());
  ChunkEntry *hcw = reinterpret_cast<ChunkEntry *>(meta.data() + (off_cws - off_pairs));
  ChunkEntry *hco = reinterpret_cast<ChunkEntry *>(meta.data() + (off_cout - off_pairs));
  XformEntry *hxf = reinterpret_cast<XformEntry *>(meta.data() + (off_xf - off_pairs));
  uint32_t *ws_dev = reinterpret_cast<uint32_t *>(pl->arena);
  size_t woff = 0, cw_i = 0, co_i = 0;
  for (size_t i = 0; i < n; ++i) {
    const hntt_poly_desc &d = descs[i];
    hp[i] = PolyPair{d.a, d.b, d.out, d.na, d.nb, (uint32_t)logs[i], 0, woff};
    woff += 6ull << logs[i];
  }
  // chunk lists grouped by length class, so that each class's chunks are one range
  for (ClassWork &cw : classes) {
    cw.ws0 = (int)cw_i;
    cw.out0 = (int)co_i;
    for (size_t i = 0; i < n; ++i) {
      if (logs[i] != cw.l) continue;
      const hntt_poly_desc &d = descs[i];
      hp[i].chunk0 = (uint32_t)co_i;
      for (uint64_t s = 0; s < (1ull << cw.l) / 2; s += kChunkWords) hcw[cw_i++] = ChunkEntry{(uint32_t)i, (uint32_t)s};
      const uint64_t nout = (uint64_t)d.na + d.nb - (big ? 0 : 1);
      for (uint64_t s = 0; s < nout; s += kChunkWords) hco[co_i++] = ChunkEntry{(uint32_t)i, (uint32_t)s};
    }
    cw.ws1 = (int)cw_i;
    cw.out1 = (int)co_i;
  }
  // transform tables per length class: forward over A_k, forward over B_k, inverse over A_k
  size_t xi = 0;
  const XformEntry *dxf = reinterpret_cast<const XformEntry *>(pl->arena + off_xf);
  for (ClassWork &cw : classes) {
    for (int half = 0; half < 2; ++half) {
      const size_t f0 = xi;
      for (size_t i = 0; i < n; ++i) {
        if (logs[i] != cw.l) continue;
        const uint64_t L = 1ull << cw.l;
        for (int k = 0; k < 3; ++k)
          hxf[xi++] = XformEntry{reinterpret_cast<uint64_t>(ws_dev + hp[i].ws_off + (2 * k + half) * L), (uint32_t)k, 0};
      }
      (half ? cw.fwd_b : cw.fwd_a) = dxf + f0;
      cw.nfwd = (int)(xi - f0);
    }
    const size_t i0 = xi;
    for (size_t i = 0; i < n; ++i) {
      if (logs[i] != cw.l) continue;
      const uint64_t L = 1ull << cw.l;
      for (int k = 0; k < 3; ++k)
        hxf[xi++] = XformEntry{reinterpret_cast<uint64_t>(ws_dev + hp[i].ws_off + (2 * k) * L), (uint32_t)k, 0};
    }
    cw.inv = dxf + i0;
    cw.ninv = (int)(xi - i0);
  }
  pl->classes = classes;

  PolyArgs &a = pl->args;
  a.pairs = reinterpret_cast<const PolyPair *>(pl->arena + off_pairs);
  a.chunks_ws = reinterpret_cast<const ChunkEntry *>(pl->arena + off_cws);
  a.nchunks_ws = (int)chunks_ws;
  a.chunks_out = reinterpret_cast<const ChunkEntry *>(pl->arena + off_cout);
  a.nchunks_out = (int)chunks_out;
  a.workspace = ws_dev;
  a.npairs = (int)n;
  a.chunk_state = reinterpret_cast<uint32_t *>(pl->arena + sz.off_state);
  a.chunk_carry = reinterpret_cast<uint32_t *>(pl->arena + sz.off_carry);
  for (int k = 0; k < 3; ++k) {
    const uint64_t q = kPrimes[k];
    const uint32_t beta = (uint32_t)((1ull << 32) % q);
    a.primes[k] = PrimeConst{(uint32_t)q, shoup32(1, q), beta, shoup32(beta, q)};
  }
  const uint64_t q1 = kPrimes[0], q2 = kPrimes[1], q3 = kPrimes[2];
  const uint64_t c12 = powmod(q1 % q2, q2 - 2, q2), c13 = powmod(q1 % q3, q3 - 2, q3),
                 c23 = powmod(q2 % q3, q3 - 2, q3);
  a.crt = CrtConst{(uint32_t)c12, shoup32(c12, q2), (uint32_t)c13, shoup32(c13, q3), (uint32_t)c23, shoup32(c23, q3)};
  a.q12 = q1 * q2;

  // upload the metadata in stream order (the copy is staged before this call returns)
  hipError_t e = hipMemcpyAsync(pl->arena + off_pairs, meta.data(), meta.size(), hipMemcpyHostToDevice,
                                (hipStream_t)stream);
  if (e != hipSuccess) {
    int r = hip_err(ctx, e, "hipMemcpyAsync(polymul metadata)");
    hntt_polymul_plan_destroy(pl.release());
    return r;
  }
  // The static form's plan lives for one call: its host image stays with the
  // context until the next such call.
  if (no_alloc) ctx->static_meta.swap(meta);
  *out = pl.release();
  return HNTT_OK;
}

static std::vector<hntt_poly_desc> as_poly(const hntt_bigmul_desc *descs, size_t n) {
  std::vector<hntt_poly_desc> v(n);
  for (size_t i = 0; i < n; ++i) v[i] = hntt_poly_desc{descs[i].a, descs[i].b, (uint64_t *)descs[i].out, descs[i].na,
                                                        descs[i].nb};
  return v;
}

extern "C" {

int hntt_polymul_plan_create(hntt_ctx *ctx, const hntt_poly_desc *descs, size_t n, uint32_t flags, void *workspace,
                             size_t workspace_bytes, void *stream, hntt_polymul_plan **out) {
  return plan_create(ctx, descs, n, flags, false, workspace, workspace_bytes, stream, out);
}

int hntt_bigmul_plan_create(hntt_ctx *ctx, const hntt_bigmul_desc *descs, size_t n, uint32_t flags, void *workspace,
                            size_t workspace_bytes, void *stream, hntt_polymul_plan **out) {
  if (ctx && n && !descs) {
    ctx->last_error = "descs is NULL";
    return HNTT_EINVAL;
  }
  const std::vector<hntt_poly_desc> pd = as_poly(descs, n);
  return plan_create(ctx, pd.data(), n, flags, true, workspace, workspace_bytes, stream, out);
}

int hntt_bigmul_workspace_size(const hntt_bigmul_desc *descs, size_t n, size_t *bytes_out) {
  if (!bytes_out || (n && !descs)) return HNTT_EINVAL;
  const std::vector<hntt_poly_desc> pd = as_poly(descs, n);
  Sizing sz;
  int rc = size_batch(nullptr, pd.data(), n, false, &sz, true);
  if (rc) return rc;
  *bytes_out = n ? sz.total : 0;
  return HNTT_OK;
}

size_t hntt_polymul_plan_workspace_bytes(const hntt_polymul_plan *plan) { return plan ? plan->arena_bytes : 0; }

int hntt_polymul_workspace_size(const hntt_poly_desc *descs, size_t n, size_t *bytes_out) {
  if (!bytes_out || (n && !descs)) return HNTT_EINVAL;
  Sizing sz;
  int rc = size_batch(nullptr, descs, n, false, &sz);
  if (rc) return rc;
  *bytes_out = n ? sz.total : 0;
  return HNTT_OK;
}

int hntt_polymul_plan_execute(hntt_ctx *ctx, hntt_polymul_plan *pl, void *stream) {
  if (!ctx || !pl || pl->ctx != ctx) return HNTT_EINVAL;
  ctx->last_error.clear();
  if (pl->n == 0) return HNTT_OK;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(ctx->device) != hipSuccess) return perr(ctx, HNTT_EDEVICE, "hipSetDevice failed");
  struct Restore {
    int d;
    ~Restore() {
      if (d >= 0) (void)hipSetDevice(d);
    }
  } restore{prev};
  hipStream_t s = (hipStream_t)stream;
  const bool use_graph = !(pl->flags & HNTT_NO_GRAPH) && !pl->graph_failed && !ctx->trace;
  if (!use_graph) {
    pl->exec_mode = pl->graph_failed ? HNTT_EXEC_CAPTURE_FAILED : HNTT_EXEC_DIRECT;
    return enqueue_plan(pl, s);
  }
  if (!pl->exec) {
    // record every launch once on a private stream (the length classes on branch
    // streams forked from it), then replay the graph on the caller's stream
    hipStream_t cs = nullptr;
    hipStream_t bs[kGraphBranches] = {};
    hipEvent_t fork[kGraphBranches] = {}, join[kGraphBranches] = {};
    const char *step = "hipStreamCreateWithFlags";
    hipError_t he = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    for (int b = 0; b < kGraphBranches && he == hipSuccess; ++b) {
      he = hipStreamCreateWithFlags(&bs[b], hipStreamNonBlocking);
      if (he == hipSuccess) he = hipEventCreateWithFlags(&fork[b], hipEventDisableTiming);
      if (he == hipSuccess) he = hipEventCreateWithFlags(&join[b], hipEventDisableTiming);
    }
    if (he == hipSuccess) {
      step = "hipStreamBeginCapture";
      he = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    }
    int rc = HNTT_OK;
    hipGraph_t g = nullptr;
    if (he == hipSuccess) {
      rc = enqueue_plan(pl, cs, Branches{bs, fork, join, kGraphBranches});
      step = "hipStreamEndCapture";
      he = hipStreamEndCapture(cs, &g);
      if (he == hipSuccess && rc != HNTT_OK) step = "enqueue under capture";
    }
    if (he == hipSuccess && rc == HNTT_OK) {
      step = "hipGraphInstantiate";
      he = hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0);
    }
    for (int b = 0; b < kGraphBranches; ++b) {
      if (fork[b]) (void)hipEventDestroy(fork[b]);
      if (join[b]) (void)hipEventDestroy(join[b]);
      if (bs[b]) (void)hipStreamDestroy(bs[b]);
    }
    if (cs) (void)hipStreamDestroy(cs);
    if (he != hipSuccess || rc != HNTT_OK) {
      // launch directly from now on, and say why (hntt_polymul_plan_exec_mode)
      pl->graph_error = std::string(step) + ": " +
                        (he != hipSuccess ? hipGetErrorString(he) : ctx->last_error.c_str());
      if (g) (void)hipGraphDestroy(g);
      pl->exec = nullptr;
      pl->graph_failed = true;
      (void)hipGetLastError();
      ctx->last_error.clear();
      pl->exec_mode = HNTT_EXEC_CAPTURE_FAILED;
      return enqueue_plan(pl, s);
    }
    pl->graph = g;
  }
  pl->exec_mode = HNTT_EXEC_GRAPH;
  return hip_err(ctx, hipGraphLaunch(pl->exec, s), "hipGraphLaunch(polymul)");
}

int hntt_polymul_plan_exec_mode(const hntt_polymul_plan *pl, const char **msg) {
  if (!pl) return HNTT_EINVAL;
  if (msg) *msg = pl->graph_error.c_str();
  return pl->exec_mode;
}

void hntt_polymul_plan_destroy(hntt_polymul_plan *pl) {
  if (!pl) return;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->owns_arena && pl->arena) {
    (void)hipFree(pl->arena);
    if (pl->ctx && pl->ctx->bytes_held >= pl->arena_bytes) pl->ctx->bytes_held -= pl->arena_bytes;
  }
  delete pl;
}

}  // extern "C"

// One-shot form shared by polynomial and large-integer products: reuse the cached
// plan when the same products are requested again (e.g. a benchmark loop).
static int one_shot(hntt_ctx *ctx, const hntt_poly_desc *descs, size_t n, uint32_t flags, bool big, void *stream) {
  hntt_polymul_plan *pl = ctx->poly_cache;
  const bool same = pl && pl->flags == flags && pl->big == big && pl->n == n &&
                    std::memcmp(pl->descs.data(), descs, n * sizeof(hntt_poly_desc)) == 0;
  if (!same) {
    if (pl) {
      (void)hipStreamSynchronize((hipStream_t)stream);  // the old plan's work may still use its arena
      hntt_polymul_plan_destroy(pl);
      ctx->poly_cache = nullptr;
    }
    int rc = plan_create(ctx, descs, n, flags, big, nullptr, 0, stream, &pl);
    if (rc) return rc;
    ctx->poly_cache = pl;
  }
  return hntt_polymul_plan_execute(ctx, pl, stream);
}

extern "C" {

int hntt_polymul_crt(hntt_ctx *ctx, const hntt_poly_desc *descs, size_t n, uint32_t flags, void *stream) {
  if (!ctx) return HNTT_EINVAL;
  ctx->last_error.clear();
  if (n == 0) return HNTT_OK;
  if (!descs) return perr(ctx, HNTT_EINVAL, "descs is NULL");
  return one_shot(ctx, descs, n, flags, false, stream);
}

int hntt_polymul_crt_static(hntt_ctx *ctx, const hntt_poly_desc *descs, size_t n, uint32_t flags, void *stream) {
  if (!ctx) return HNTT_EINVAL;
  ctx->last_error.clear();
  if (n == 0) return HNTT_OK;
  if (!descs) return perr(ctx, HNTT_EINVAL, "descs is NULL");
  if (flags & ~(HNTT_PLAIN | HNTT_NO_GRAPH)) return perr(ctx, HNTT_EINVAL, "unknown flag bits");
  // the size is known from the lengths: an oversized batch fails before the device is touched
  Sizing sz;
  int rc = size_batch(ctx, descs, n, true, &sz);
  if (rc) return rc;
  if (sz.total > kStaticScratchBytes)
    return perr(ctx, HNTT_ENOMEM, "batch needs %zu bytes of workspace; the static workspace holds %zu", sz.total,
                kStaticScratchBytes);
  if ((rc = ensure_device(ctx))) return rc;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (hipSetDevice(ctx->device) != hipSuccess) return perr(ctx, HNTT_EDEVICE, "hipSetDevice failed");
  struct Restore {
    int d;
    ~Restore() {
      if (d >= 0) (void)hipSetDevice(d);
    }
  } restore{prev};
  void *ws = nullptr;
  hipError_t e = static_scratch_address(ctx->device, &ws);
  if (e != hipSuccess) return hip_err(ctx, e, "address of the static workspace");
  hntt_polymul_plan *pl = nullptr;
  rc = plan_create(ctx, descs, n, flags | HNTT_NO_GRAPH, false, ws, kStaticScratchBytes, stream, &pl, true);
  if (rc) return rc;
  rc = enqueue_plan(pl, (hipStream_t)stream);
  hntt_polymul_plan_destroy(pl);  // host bookkeeping only: the workspace is not the plan's
  return rc;
}

int hntt_bigmul(hntt_ctx *ctx, const hntt_bigmul_desc *descs, size_t n, uint32_t flags, void *stream) {
  if (!ctx) return HNTT_EINVAL;
  ctx->last_error.clear();
  if (n == 0) return HNTT_OK;
  if (!descs) return perr(ctx, HNTT_EINVAL, "descs is NULL");
  const std::vector<hntt_poly_desc> pd = as_poly(descs, n);
  return one_shot(ctx, pd.data(), n, flags, true, stream);
}

}  // extern "C"

void hntt_ctx::release_poly_cache() {
  if (poly_cache) {
    hntt_polymul_plan_destroy(poly_cache);
    poly_cache = nullptr;
  }
}
