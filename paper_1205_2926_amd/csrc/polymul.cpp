// Exact polynomial products through three NTT primes and Chinese remaindering.
#include "hntt.h"
#include "hntt_internal.hpp"

extern "C" int hntt_polymul_crt(hntt_ctx *ctx, const hntt_poly_desc *descs, size_t n, uint32_t flags, void *stream) {
  (void)descs; (void)n; (void)flags; (void)stream;
  if (!ctx) return HNTT_EINVAL;
  ctx->last_error = "hntt_polymul_crt is not built yet";
  return HNTT_EUNSUPPORTED;
}
