// Device-side records and launchers of the three-prime polynomial product.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hntt {

// One product of the batch.  Its workspace (ws_off words into the plan's arena)
// holds six arrays of L = 2^log2_len words: A1, B1, A2, B2, A3, B3 (operands
// reduced mod q_k, zero-padded, transformed in place; A_k ends as the residues
// of the product mod q_k).
struct PolyPair {
  const uint32_t *a;
  const uint32_t *b;
  void *out;           // uint64_t coefficients, or (large-integer mode) uint32_t limbs
  uint32_t na, nb;
  uint32_t log2_len;
  uint32_t chunk0;     // large-integer mode: index of the product's first output chunk
  uint64_t ws_off;
};

// A 1024-word chunk of one product's positions.
struct ChunkEntry {
  uint32_t pair;
  uint32_t start;
};

// Per-prime constants: q, floor(2^32/q) (Shoup constant of 1), q^-1 mod 2^32,
// 2^64 mod q.
struct PrimeConst {
  uint32_t q, one_p;    // q and floor(2^32 / q) (Shoup constant of 1)
  uint32_t beta, beta_p;  // 2^32 mod q and its Shoup constant
};

// Garner constants with their Shoup constants: q1^-1 mod q2, q1^-1 mod q3, q2^-1 mod q3.
struct CrtConst {
  uint32_t c12, c12p, c13, c13p, c23, c23p;
};

struct PolyArgs {
  const PolyPair *pairs;
  const ChunkEntry *chunks_ws;   // chunks over the lower half (L / 2 words) of every product
  int nchunks_ws;
  const ChunkEntry *chunks_out;  // chunks over the na + nb - 1 output coefficients
                                 // (large-integer mode: over the na + nb limbs)
  int nchunks_out;
  int npairs;
  uint32_t *workspace;
  PrimeConst primes[3];
  CrtConst crt;
  // Large-integer mode (products of base-2^32 limb integers): q1 q2, and per
  // output chunk its carry state (kill / generate / propagate) and carry-in.
  uint64_t q12;
  uint32_t *chunk_state;
  uint32_t *chunk_carry;
};

hipError_t launch_poly_prep(const PolyArgs &a, hipStream_t s);
hipError_t launch_poly_crt(const PolyArgs &a, hipStream_t s);
// Large-integer mode: exact coefficients as three 32-bit words each (Garner,
// written over the dead B_k arrays of the workspace), then the carry pass that
// turns them into na + nb limbs at PolyPair::out.
hipError_t launch_big_crt(const PolyArgs &a, hipStream_t s);
hipError_t launch_big_carry(const PolyArgs &a, hipStream_t s);

}  // namespace hntt
