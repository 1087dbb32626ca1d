/*
 * hntt — lazy-butterfly number-theoretic transforms on AMD MI355X (gfx950).
 *
 * C ABI of the GPU library.  It implements the radix-2 NTT over F_p of
 * D. Harvey, "Faster arithmetic for number-theoretic transforms"
 * (arXiv:1205.2926), for word-sized primes p = 1 (mod L), L = 2^l:
 *
 *   forward   b_j = sum_{i<L} omega^(ij) a_i  (mod p)           Section 1, display eq.
 *             natural-order input, output in bit-reversed order  Section 1, Algorithm 1
 *   inverse   a_i = L^(-1) sum_{j<L} omega^(-ij) b_j  (mod p)
 *             bit-reversed input, natural-order output           Section 4 (Algorithm 1 run backwards)
 *
 * The default butterflies are the lazy ones: Algorithm 3 (forward, residues
 * kept in [0,2p)) and Algorithm 4 (inverse, residues kept in [0,4p)), each
 * multiplying by a precomputed Shoup constant W' = floor(W beta / p).  The
 * flag HNTT_PLAIN selects the fully reducing butterfly of Algorithm 2 (and its
 * inverse counterpart) under the same kernel schedule, for comparison; the
 * flag HNTT_MONT selects the Montgomery butterfly of Algorithm 5 (and the
 * inverse butterfly of Algorithm 4 with Montgomery's product), whose tables
 * hold only W beta mod p per root.
 *
 * Conventions shared by every entry point
 *   - Return value: HNTT_OK (0) or a negative HNTT_E* status.  Nothing throws.
 *   - Argument errors (HNTT_EINVAL, HNTT_EUNSUPPORTED) are found on the host
 *     before anything is enqueued: on such a return no device work was issued.
 *   - Data buffers are DEVICE pointers owned by the caller; descriptor arrays
 *     are HOST memory, read during the call and not retained.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*, NULL = the
 *     default stream) and runs asynchronously in stream order.  A device
 *     failure is reported as HNTT_EDEVICE by the failing call or a later one.
 *   - Inputs must be fully reduced residues in [0,p); outputs are fully
 *     reduced to [0,p) (bit-exact with any correct implementation).
 *   - A context is used by one host thread at a time.
 *   - hntt_last_error(ctx) returns a human-readable message for the most
 *     recent failure on that context.
 */
#ifndef HNTT_H
#define HNTT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HNTT_OK = 0,
  HNTT_EINVAL = -1,       /* malformed argument or descriptor */
  HNTT_EUNSUPPORTED = -2, /* well-formed but outside what the library implements */
  HNTT_ENOMEM = -3,       /* device memory (or the context's memory budget) exhausted */
  HNTT_EDEVICE = -4,      /* HIP runtime or device error */
  HNTT_EBUSY = -5         /* serving: request cannot be admitted now */
};

/* Flags for the transform entry points. */
#define HNTT_PLAIN 0x1u        /* fully reducing butterflies (Algorithm 2 and its DIT twin) */
#define HNTT_NO_NORMALIZE 0x2u /* skip the final reduction: forward leaves [0,2p) (lazy),
                                  inverse leaves [0,4p) (lazy); for chained pipelines only */
#define HNTT_MONT 0x8u         /* Montgomery butterflies: Algorithm 5 (Section 4) forward and
                                  Algorithm 4 with Montgomery's product inverse; tables hold
                                  one word W beta mod p per root; same ranges and bounds as lazy */
#define HNTT_VALIDATE 0x10u    /* check on the device that every input word is below p (the
                                  [0,p) precondition of the transforms and of the pointwise
                                  product) before anything else is enqueued: an input outside
                                  it fails the call with EINVAL naming the first such
                                  descriptor, and no data is changed.  The check waits for the
                                  stream (a host synchronisation), so it cannot be used while
                                  the stream is being captured into a graph. */

typedef struct hntt_ctx hntt_ctx;

/* Create a context bound to HIP device `device`.  The device is touched only
 * when the first computation is enqueued, so argument checking works without
 * a GPU.  `mem_budget_bytes` caps the device memory the context may hold for
 * twiddle tables and polynomial workspaces (0 = no cap).
 * Errors: EINVAL (out == NULL or device < 0), ENOMEM (host allocation). */
int hntt_create(hntt_ctx **out, int device, size_t mem_budget_bytes);

/* Free the context and every device buffer it owns.  NULL is ignored.  The
 * caller must make sure no enqueued work still uses the context. */
void hntt_destroy(hntt_ctx *ctx);

/* Static description of a status code. */
const char *hntt_strerror(int status);

/* Message of the last failure on ctx ("" if none).  Valid until the next call on ctx. */
const char *hntt_last_error(const hntt_ctx *ctx);

/* One transform: `data` is a device array of 2^log2_len words of word_bits
 * bits (32: uint32_t, 64: uint64_t), transformed in place, aligned to 16
 * bytes (or to its size, if that is smaller).
 *   p        prime, p = 1 (mod 2^log2_len).  Lazy and Montgomery butterflies
 *            need p < beta/4 (Algorithm 3 and 5 input conditions); HNTT_PLAIN
 *            needs p < beta/2 (Algorithm 2 input conditions); beta = 2^word_bits.
 *   omega    a primitive 2^log2_len-th root of unity mod p (Section 1): the
 *            transform is defined by it, another root permutes the output.
 *   log2_len 1 <= l <= 30 (and 2^l words must be addressable).
 * Primality of p is checked once per context with deterministic Miller-Rabin;
 * omega is checked by omega^(L/2) = p - 1. */
typedef struct {
  uint64_t p;
  uint64_t omega;
  void *data;
  uint32_t log2_len;
  uint32_t word_bits;
} hntt_desc;

/* Forward NTT of n descriptors (Section 1, Algorithm 1 with the Algorithm 3
 * butterfly).  Natural-order input in [0,p), bit-reversed output in [0,p).
 * Descriptors may mix primes, lengths and word sizes; descriptors that share
 * (p, omega, log2_len, word_bits) are transformed by the same launches.
 * Two descriptors must not name overlapping data.  flags: HNTT_PLAIN or
 * HNTT_MONT (not both: EINVAL), HNTT_NO_NORMALIZE, HNTT_VALIDATE.
 * Errors: EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE. */
int hntt_ntt_forward(hntt_ctx *ctx, const hntt_desc *descs, size_t n, uint32_t flags, void *stream);

/* Inverse NTT (Section 4: Algorithm 1 run backwards with the Algorithm 4
 * butterfly, then multiplication by L^(-1)).  Bit-reversed input in [0,p),
 * natural-order output in [0,p); inverse(forward(x)) = x.  Same descriptor
 * rules, flags and errors as hntt_ntt_forward. */
int hntt_ntt_inverse(hntt_ctx *ctx, const hntt_desc *descs, size_t n, uint32_t flags, void *stream);

/* Pointwise product c_i = a_i b_i (mod p) over `len` words of word_bits bits
 * (device pointers; c may alias a or b).  Needs p < 2^31 for 32-bit words and
 * p < 2^62 for 64-bit words; inputs in [0,p), output in [0,p).  Used between
 * forward and inverse transforms to multiply polynomials (the convolution
 * theorem behind the application named in Section 1).  flags: 0 or
 * HNTT_VALIDATE (checks a and b).
 * Errors: EINVAL, EUNSUPPORTED, EDEVICE. */
typedef struct {
  uint64_t p;
  const void *a;
  const void *b;
  void *c;
  uint64_t len;
  uint32_t word_bits;
  uint32_t reserved; /* must be 0 */
} hntt_pw_desc;
int hntt_pointwise_mul(hntt_ctx *ctx, const hntt_pw_desc *descs, size_t n, uint32_t flags, void *stream);

/* Exact integer polynomial products (the application named in Section 1)
 * through three NTT primes, q1 = 998244353, q2 = 754974721, q3 = 167772161, and
 * Chinese remaindering (Garner).  For each descriptor: a has na >= 1 and b has
 * nb >= 1 uint32 coefficients (device, 4-byte aligned), out receives the
 * na + nb - 1 coefficients of a*b as uint64 (device, 8-byte aligned).  Each
 * product is zero-padded to L = 2 * nextpow2(max(na, nb)) <= 2^23 and
 * computed as forward NTTs of a and b mod each q_k, a pointwise product, an
 * inverse NTT, and CRT.  The result is the exact integer when every product
 * coefficient is below 2^64 (it is always below q1 q2 q3 ~ 2^86.7 for
 * coefficients below 2^20 and min(na, nb) <= 2^23; it is then returned mod
 * 2^64 if it exceeds 2^64).  Products of any mix of lengths run together: the
 * lengths are grouped into classes, each class's transforms for all three
 * primes go through the same pass launches (per-transform prime slots), and
 * operand preparation, pointwise products and CRT run as persistent kernels
 * over the whole batch.
 * flags: HNTT_PLAIN (fully reducing butterflies), HNTT_NO_GRAPH (enqueue the
 * kernels directly instead of replaying a recorded HIP graph); HNTT_MONT is
 * not accepted here (EINVAL).
 * Errors: EINVAL (NULL/misaligned pointer, empty operand), EUNSUPPORTED
 * (padded length above 2^23), ENOMEM, EDEVICE. */
typedef struct {
  const uint32_t *a;
  const uint32_t *b;
  uint64_t *out;
  uint32_t na;
  uint32_t nb;
} hntt_poly_desc;

#define HNTT_NO_GRAPH 0x4u

/* One-shot form: plans (reusing the previous plan of this context when the
 * descriptors are identical) and executes on `stream`.  The context owns the
 * plan's workspace. */
int hntt_polymul_crt(hntt_ctx *ctx, const hntt_poly_desc *descs, size_t n, uint32_t flags, void *stream);

/* Plan / execute form, for callers that keep several batches in flight.
 * hntt_polymul_plan_create checks the descriptors on the host, builds the
 * twiddle tables it needs (cached on the context), lays out the workspace and
 * uploads the plan's metadata on `stream`.  The workspace is either supplied by
 * the caller (`workspace`, `workspace_bytes`: device memory, 256-byte aligned,
 * at least hntt_polymul_plan_workspace_bytes of the plan — pass NULL first to
 * learn the size) or allocated by the plan (workspace = NULL).  The descriptor
 * pointers are captured: the operands must stay valid until execution ends.
 * hntt_polymul_plan_execute enqueues only kernel launches (no device
 * allocation, no copies, no synchronisation).  Unless HNTT_NO_GRAPH was given,
 * the first execution records the launches into a HIP graph, on private streams
 * it creates and destroys for that (each length class on a parallel branch),
 * and every execution replays the graph on `stream`; with HNTT_NO_GRAPH the
 * kernels are launched one by one on `stream`, which is the form to use when the
 * caller itself captures the execution into a graph.  Two executions of one plan
 * must not overlap (they share the workspace).
 * hntt_polymul_plan_destroy frees what the plan owns; the caller must make sure
 * no enqueued execution still uses it.
 * Errors as for hntt_polymul_crt; ENOMEM if the given workspace is too small. */
typedef struct hntt_polymul_plan hntt_polymul_plan;
int hntt_polymul_plan_create(hntt_ctx *ctx, const hntt_poly_desc *descs, size_t n, uint32_t flags, void *workspace,
                             size_t workspace_bytes, void *stream, hntt_polymul_plan **out);
size_t hntt_polymul_plan_workspace_bytes(const hntt_polymul_plan *plan);
/* How the plan's last execution was enqueued: HNTT_EXEC_NONE (not executed yet),
 * HNTT_EXEC_GRAPH (one HIP graph launch), HNTT_EXEC_DIRECT (kernel launches, as
 * asked by HNTT_NO_GRAPH or while tracing is on), or HNTT_EXEC_CAPTURE_FAILED
 * (kernel launches because recording the graph failed; the plan keeps launching
 * directly, and msg, when not NULL, receives the reason).  Host only. */
enum { HNTT_EXEC_NONE = 0, HNTT_EXEC_GRAPH = 1, HNTT_EXEC_DIRECT = 2, HNTT_EXEC_CAPTURE_FAILED = 3 };
int hntt_polymul_plan_exec_mode(const hntt_polymul_plan *plan, const char **msg);
/* Workspace a plan for these descriptors needs, computed on the host from the
 * lengths alone (pointers are not read), e.g. for admission control before any
 * device memory is committed.  Errors: EINVAL, EUNSUPPORTED. */
int hntt_polymul_workspace_size(const hntt_poly_desc *descs, size_t n, size_t *bytes_out);
int hntt_polymul_plan_execute(hntt_ctx *ctx, hntt_polymul_plan *plan, void *stream);
void hntt_polymul_plan_destroy(hntt_polymul_plan *plan);

/* Allocation-free form of hntt_polymul_crt, for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc).  Same
 * products, descriptors and results as hntt_polymul_crt; the difference is
 * where the workspace lives and what the call may do:
 *   - the workspace (reduced, padded operands of the three primes and the
 *     batch's metadata) is a static device array of HNTT_STATIC_SCRATCH_BYTES
 *     that the library holds on every GPU it is loaded on until the process
 *     ends; a batch needing more (hntt_polymul_workspace_size) fails with
 *     ENOMEM before anything is enqueued;
 *   - the call issues no hipMalloc/hipFree and builds no twiddle table: the
 *     tables of every padded length in the batch must already be resident on
 *     ctx (made by an earlier hntt_polymul_crt or hntt_polymul_plan_create with
 *     products of the same padded lengths and flags); otherwise EUNSUPPORTED,
 *     nothing enqueued;
 *   - kernels are enqueued directly (no graph); the metadata goes to the device
 *     with one asynchronous host-to-device copy on `stream`;
 *   - every call on one GPU shares that GPU's workspace and leaves its contents
 *     there; nothing in it needs to start at zero.  Calls in stream order on one
 *     stream are safe; calls that overlap on one GPU (other streams, other
 *     contexts, other host threads) race on the workspace and give wrong
 *     results.
 * flags: HNTT_PLAIN, HNTT_NO_GRAPH (accepted, implied).
 * Errors: EINVAL, EUNSUPPORTED (padded length above 2^23, or tables not yet
 * resident), ENOMEM (batch larger than the static workspace), EDEVICE. */
#define HNTT_STATIC_SCRATCH_BYTES ((size_t)32 << 20)
int hntt_polymul_crt_static(hntt_ctx *ctx, const hntt_poly_desc *descs, size_t n, uint32_t flags, void *stream);

/* ---------------------------------------------------------------------------
 * Large-integer multiplication (the application that Section 1 names for fast
 * transforms): out = a * b for non-negative integers given as little-endian
 * base-2^32 limbs.  The limbs are the coefficients of a polynomial product
 * (hntt_polymul_*: three primes, lazy butterflies, Garner), whose exact
 * coefficients (below min(na, nb) (2^32 - 1)^2 < 2^86 < q1 q2 q3) are carried
 * into limbs on the device by a parallel carry scan.
 *   a, b   na, nb limbs (device, 4-byte aligned), 1 <= na, nb and
 *          2 * nextpow2(max(na, nb)) <= 2^23 (operands up to 2^22 limbs);
 *   out    na + nb limbs (device, 4-byte aligned, not overlapping a or b);
 *          the product always fits.
 * flags: HNTT_PLAIN, HNTT_NO_GRAPH as for hntt_polymul_crt.  The plan form
 * returns an hntt_polymul_plan, executed and destroyed with the
 * hntt_polymul_plan_* calls above; hntt_bigmul_workspace_size gives its
 * workspace from the lengths.  Errors: EINVAL (NULL/misaligned pointer, empty
 * operand), EUNSUPPORTED (operand above 2^22 limbs), ENOMEM, EDEVICE.
 * ------------------------------------------------------------------------- */
typedef struct {
  const uint32_t *a;
  const uint32_t *b;
  uint32_t *out;
  uint32_t na;
  uint32_t nb;
} hntt_bigmul_desc;
int hntt_bigmul(hntt_ctx *ctx, const hntt_bigmul_desc *descs, size_t n, uint32_t flags, void *stream);
int hntt_bigmul_plan_create(hntt_ctx *ctx, const hntt_bigmul_desc *descs, size_t n, uint32_t flags, void *workspace,
                            size_t workspace_bytes, void *stream, hntt_polymul_plan **out);
int hntt_bigmul_workspace_size(const hntt_bigmul_desc *descs, size_t n, size_t *bytes_out);

/* ---------------------------------------------------------------------------
 * Host-side number theory (no device needed).  These are the parameters of
 * the problem setting in Section 1 and the Shoup constant of Algorithm 2.
 * ------------------------------------------------------------------------- */

/* 1 if n is prime (deterministic Miller-Rabin for 64-bit n), else 0. */
int hntt_is_prime(uint64_t n);

/* Smallest primitive root of the prime p, or 0 if p is not an odd prime. */
uint64_t hntt_primitive_root(uint64_t p);

/* omega = g^((p-1)/2^log2_len) for the smallest primitive root g of p.
 * Errors: EINVAL if p is not prime or 2^log2_len does not divide p - 1. */
int hntt_root_of_unity(uint64_t p, uint32_t log2_len, uint64_t *omega_out);

/* Largest prime p < 2^bits with p = 1 (mod 2^v), 2 <= bits <= 64, v < bits;
 * 0 if none. */
uint64_t hntt_find_prime(uint32_t bits, uint32_t v);

/* Shoup constant W' = floor(W * 2^word_bits / p) for 0 <= W < p (Algorithm 2
 * input conditions).  Errors: EINVAL on W >= p, p < 2, p >= 2^word_bits. */
int hntt_shoup_constant(uint64_t w, uint64_t p, uint32_t word_bits, uint64_t *wprime_out);

/* Check descriptors as hntt_ntt_forward would, without touching the device.
 * Returns HNTT_OK or the error the transform call would return (HNTT_VALIDATE
 * is accepted; its device check of the data runs only in the transform calls). */
int hntt_validate(hntt_ctx *ctx, const hntt_desc *descs, size_t n, uint32_t flags);

/* ---------------------------------------------------------------------------
 * Schedule tuning.  A transform of length 2^l above the one-workgroup limit
 * runs as a column pass and a row pass (an R x C view, l = log R + log C): the
 * first log R stages of Algorithm 1 (Section 1) are fused into the column pass
 * and the last row_log2 = log C into the row pass.  g_cols / g_rows are the
 * sub-transforms (columns / rows) one workgroup owns in each (g_rows_inv: rows
 * per workgroup in the inverse transform's row pass, 0 meaning g_rows), and batch_chunk
 * the number of transforms that go through all passes before the next chunk
 * starts (so a chunk's intermediate result can stay in the last-level cache).
 * Fields set to 0 keep the built-in choice (row_log2: ceil(l / 2); both passes
 * must stay within 1..12 stages).  hntt_set_tuning overrides the schedule for
 * (log2_len, word_bits) on this context (EINVAL if a value does not fit the
 * kernels: powers of two, thread and LDS limits, batch_chunk <= 64);
 * hntt_get_plan reports the schedule in effect.  Results never depend on the
 * schedule; only speed does.
 * ------------------------------------------------------------------------- */
typedef struct {
  uint32_t log2_len;
  uint32_t word_bits;
  uint32_t g_cols;
  uint32_t g_rows;
  uint32_t batch_chunk;
  uint32_t row_log2;
  uint32_t g_rows_inv;
} hntt_tuning;
int hntt_set_tuning(hntt_ctx *ctx, const hntt_tuning *t);
int hntt_get_plan(hntt_ctx *ctx, uint32_t log2_len, uint32_t word_bits, hntt_tuning *out);

/* ---------------------------------------------------------------------------
 * Kernel timing (tracing).  While enabled, every kernel the context launches
 * is bracketed by two HIP events recorded on its launch stream.
 * hntt_trace_read waits for the pending events and writes, as JSON text,
 * {"<kernel>": {"launches": n, "total_ms": t}, ...} accumulated since the last
 * reset into buf (capacity *len bytes); *len receives the size needed.  Kernel
 * names are <pass>_<fwd|inv|fwdmulinv>_<lazy|plain|mont>_u<bits>_n<log2 sub-length>
 * (fwdmulinv: a product's fused forward pass, pointwise product and first
 * inverse pass) for transform passes, and poly_prep, poly_crt, big_crt and
 * big_carry for the product kernels.
 * Errors: EINVAL; ENOMEM when buf is NULL or too small; EDEVICE.
 * ------------------------------------------------------------------------- */
int hntt_trace_enable(hntt_ctx *ctx, int enable);
int hntt_trace_read(hntt_ctx *ctx, char *buf, size_t *len);
int hntt_trace_reset(hntt_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Device unit test of the butterflies themselves (Algorithms 2, 3, 4, 5).
 * kind: 0 = Algorithm 2 (plain forward), 1 = Algorithm 3 (lazy forward),
 *       2 = Algorithm 4 (lazy inverse),  3 = plain inverse (fully reducing),
 *       4 = Algorithm 5 (Montgomery forward), 5 = Montgomery lazy inverse
 *       (Algorithm 4 with the product of Algorithm 5).
 * For i < n: (xo[i], yo[i]) = butterfly(x[i], y[i]).  Kinds 0-3: w[i] is the
 * twiddle W and wprime[i] its Shoup constant floor(W beta / p); kinds 4-5: w[i]
 * is W beta mod p and wprime[i] is p^-1 mod beta.  All arrays are device arrays
 * of word_bits-bit words.  Inputs must satisfy the algorithm's stated ranges.
 * Errors: EINVAL, EUNSUPPORTED, EDEVICE.
 * ------------------------------------------------------------------------- */
int hntt_debug_butterfly(hntt_ctx *ctx, int kind, uint32_t word_bits, uint64_t p, const void *x,
                         const void *y, const void *w, const void *wprime, void *xo, void *yo, size_t n,
                         void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HNTT_H */
