// Word-size modular arithmetic for the RNS limbs of the BFV ciphertext ring.
//
// Every prime p used on the GPU lies in (2^53, 2^54) and satisfies
// p = 1 mod 2N (negacyclic NTT-friendly); t = 65537 is handled separately.
// Residues are kept as uint64 in [0, p) at kernel boundaries; inside the NTT
// butterflies they are lazy (below 57p in the forward transform, below
// 2^4 4p within an inverse pass), always below 2^61.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PEPSI_HD __host__ __device__ __forceinline__

typedef unsigned __int128 u128;

// High 64 bits of a 64x64 product.
PEPSI_HD uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((u128)a * b) >> 64);
#endif
}

// Per-prime constants.
struct Prime {
  uint64_t p;
  uint64_t barrett;   // floor(2^116 / p)  (< 2^63 for p > 2^53)
  uint64_t r64;       // 2^64 mod p
};

// w * x mod p with the Shoup companion wq = floor(w 2^64 / p); x < 2^64, w < p.
// Result in [0, 2p).
PEPSI_HD uint64_t shoup_lazy(uint64_t x, uint64_t w, uint64_t wq, uint64_t p) {
  uint64_t q = mulhi64(x, wq);
  return x * w - q * p;
}
// As shoup_lazy, with the quotient taken from the three partial products of x wq that reach its
// top word: the low halves of the two cross products and all of the lowest product are dropped,
// so the quotient is at most 2 short and the result lies in [0, 4p). The product is formed mod
// 2^64 from 32-bit halves as x w + q (2^64 - p): three 32 x 32 -> 64 multiply-adds for the low
// word, and the high word collects the four cross products' low halves. The empty asm keeps the
// halves of x opaque, so that the compiler does not fold them back into a 64-bit multiply.
PEPSI_HD uint64_t shoup_lazy4(uint64_t x, uint64_t w, uint64_t wq, uint64_t p) {
  uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
#if defined(__HIP_DEVICE_COMPILE__)
  __asm__("" : "+v"(x0), "+v"(x1));
#endif
  const uint32_t c0 = (uint32_t)wq, c1 = (uint32_t)(wq >> 32);
  const uint64_t hs = (((uint64_t)x1 * c0) >> 32) + (((uint64_t)x0 * c1) >> 32);
  const uint64_t q = (uint64_t)x1 * c1 + hs;
  const uint64_t n = 0 - p;
  const uint32_t w0 = (uint32_t)w, w1 = (uint32_t)(w >> 32), n0 = (uint32_t)n, n1 = (uint32_t)(n >> 32);
  const uint32_t q0 = (uint32_t)q, q1 = (uint32_t)(q >> 32);
  uint64_t r = (uint64_t)x0 * w0;
  r += (uint64_t)q0 * n0;
  const uint32_t hi = (uint32_t)(r >> 32) + x1 * w0 + x0 * w1 + q1 * n0 + q0 * n1;
  return ((uint64_t)hi << 32) | (uint32_t)r;
}
PEPSI_HD uint64_t shoup(uint64_t x, uint64_t w, uint64_t wq, uint64_t p) {
  uint64_t r = shoup_lazy(x, w, wq, p);
  return r >= p ? r - p : r;
}
PEPSI_HD uint64_t shoup_companion(uint64_t w, uint64_t p) {
  return (uint64_t)(((u128)w << 64) / p);
}

// x mod p for x = hi:lo < 2^116 (Barrett with the quotient estimated from
// x >> 52; the estimate is at most 2 short, so two corrections suffice).
// The same without the corrections: congruent to x and below 3p.
PEPSI_HD uint64_t reduce116_lazy(uint64_t lo, uint64_t hi, const Prime& P) {
  uint64_t top = (lo >> 52) | (hi << 12);          // floor(x / 2^52) < 2^64
  uint64_t q = mulhi64(top, P.barrett);            // ~ floor(x / p)
  return lo - q * P.p;                             // true remainder + k p, k in {0,1,2}
}
PEPSI_HD uint64_t reduce116(uint64_t lo, uint64_t hi, const Prime& P) {
  uint64_t r = reduce116_lazy(lo, hi, P);
  if (r >= P.p) r -= P.p;
  if (r >= P.p) r -= P.p;
  return r;
}
// x mod p for any 128-bit x: fold the top word first (hi * 2^64 = (hi mod p) * r64).
PEPSI_HD uint64_t reduce128(uint64_t lo, uint64_t hi, const Prime& P) {
  if (hi >> 52) {
    u128 f = (u128)(hi % P.p) * P.r64 + lo;          // < 2^108 + 2^64
    return reduce116((uint64_t)f, (uint64_t)(f >> 64), P);
  }
  return reduce116(lo, hi, P);
}
PEPSI_HD uint64_t mulmod(uint64_t a, uint64_t b, const Prime& P) {
  u128 x = (u128)a * b;
  return reduce116((uint64_t)x, (uint64_t)(x >> 64), P);
}
// Congruent to a b and below 3p, for a b < 2^116.
PEPSI_HD uint64_t mulmod_lazy(uint64_t a, uint64_t b, const Prime& P) {
  u128 x = (u128)a * b;
  return reduce116_lazy((uint64_t)x, (uint64_t)(x >> 64), P);
}
PEPSI_HD uint64_t addmod(uint64_t a, uint64_t b, uint64_t p) {
  uint64_t s = a + b;
  return s >= p ? s - p : s;
}
PEPSI_HD uint64_t submod(uint64_t a, uint64_t b, uint64_t p) {
  return a >= b ? a - b : a + p - b;
}

// ---- the plaintext modulus t = 65537 = 2^16 + 1 ----
#define PEPSI_T 65537u
PEPSI_HD uint32_t mod_t(uint64_t x) { return (uint32_t)(x % PEPSI_T); }
PEPSI_HD uint32_t mulmod_t(uint32_t a, uint32_t b) { return mod_t((uint64_t)a * b); }
PEPSI_HD uint32_t addmod_t(uint32_t a, uint32_t b) {
  uint32_t s = a + b;
  return s >= PEPSI_T ? s - PEPSI_T : s;
}
PEPSI_HD uint32_t submod_t(uint32_t a, uint32_t b) {
  return a >= b ? a - b : a + PEPSI_T - b;
}
