// Device helpers shared by the kernels: GF(2^61-1) arithmetic for the
// CountSketch signs, the Philox4x32-10 counter-based generator and the
// Box-Muller transform.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lev_internal.h"

namespace lev {

constexpr uint64_t kP61 = (1ull << 61) - 1;

// (x * y) mod (2^61 - 1) for x, y < 2^61.  The 122-bit product is folded
// with 2^61 = 1 (mod p61).
__device__ __forceinline__ uint64_t mulmod_p61(uint64_t x, uint64_t y) {
  const uint64_t lo = x * y;
  const uint64_t hi = __umul64hi(x, y);
  uint64_t r = (lo & kP61) + ((lo >> 61) | (hi << 3));
  r = (r & kP61) + (r >> 61);
  return r >= kP61 ? r - kP61 : r;
}

__device__ __forceinline__ uint64_t addmod_p61(uint64_t x, uint64_t y) {
  uint64_t r = x + y;  // < 2^62
  r = (r & kP61) + (r >> 61);
  return r >= kP61 ? r - kP61 : r;
}

// CountSketch sign of row i: +1 if g(i) is even, g the cubic of HashParams.
__device__ __forceinline__ bool sign_negative(const HashParams& hp, uint64_t i) {
  uint64_t g = hp.c3;
  g = addmod_p61(mulmod_p61(g, i), hp.c2);
  g = addmod_p61(mulmod_p61(g, i), hp.c1);
  g = addmod_p61(mulmod_p61(g, i), hp.c0);
  return (g & 1ull) != 0;
}

// x mod P for any 64-bit x (P < 2^32), by Barrett reduction with
// pbar = floor((2^64 - 1) / P): the quotient estimate umulhi(x, pbar) is at
// most two below floor(x / P), so two conditional subtractions finish it
// (a 64-bit division is a long software sequence on the GPU).
__device__ __forceinline__ uint64_t mod_p(const HashParams& hp, uint64_t x) {
  uint64_t r = x - __umul64hi(x, hp.pbar) * hp.P;
  r = r >= hp.P ? r - hp.P : r;
  return r >= hp.P ? r - hp.P : r;
}

// Bucket-hash argument of row i: (a i + c) mod P (a, i, c < P < 2^32, so
// a i + c < 2^64).
__device__ __forceinline__ uint64_t hash_x(const HashParams& hp, uint64_t i) {
  return mod_p(hp, hp.a * i + hp.c);
}

// Row id at position t of bucket b's progression: (i0 + t*delta) mod P.
// P < 2^32 and t, delta < 2^32, so t*delta fits in 64 bits.
__device__ __forceinline__ uint64_t bucket_row(const HashParams& hp, uint64_t i0, uint64_t t) {
  const uint64_t r = i0 + mod_p(hp, t * hp.delta);  // < 2 P
  return r >= hp.P ? r - hp.P : r;
}

__device__ __forceinline__ uint64_t bucket_start(const HashParams& hp, int64_t b) {
  const uint64_t x = (uint64_t)b;  // b < P here
  const uint64_t diff = mod_p(hp, x + hp.P - hp.c);
  return mod_p(hp, hp.ainv * diff);
}

__device__ __forceinline__ int64_t bucket_len(const HashParams& hp, int64_t b) {
  const int64_t P = (int64_t)hp.P;
  return b < P ? (P - b + hp.r_cs - 1) / hp.r_cs : 0;
}

// ---- Philox4x32-10 (Salmon et al., SC 2011) ----
struct U32x4 {
  uint32_t x0, x1, x2, x3;
};

__device__ __forceinline__ U32x4 philox4x32_10(U32x4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const uint32_t lo0 = M0 * c.x0, hi0 = __umulhi(M0, c.x0);
    const uint32_t lo1 = M1 * c.x2, hi1 = __umulhi(M1, c.x2);
    c = U32x4{hi1 ^ c.x1 ^ k0, lo1, hi0 ^ c.x3 ^ k1, lo0};
  }
  return c;
}

// Two N(0,1) values (cosine and sine branch) from one Philox counter.
__device__ __forceinline__ void box_muller_pair(uint64_t counter, PhiloxKey key, double* z_even,
                                                double* z_odd) {
  const U32x4 x = philox4x32_10(U32x4{(uint32_t)counter, (uint32_t)(counter >> 32), 0u, 0u},
                                key.k0, key.k1);
  const uint64_t a = ((uint64_t)x.x0 << 21) | ((uint64_t)x.x1 >> 11);
  const uint64_t b = ((uint64_t)x.x2 << 21) | ((uint64_t)x.x3 >> 11);
  const double u1 = ((double)a + 0.5) * 0x1.0p-53;
  const double u2 = ((double)b + 0.5) * 0x1.0p-53;
  const double radius = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);  // sin, cos of 2 pi u2; 2 u2 is exact, so no reduction by pi is needed
  *z_even = radius * cs;
  *z_odd = radius * sn;
}

}  // namespace lev
