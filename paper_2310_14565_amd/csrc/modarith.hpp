// Word-size modular arithmetic for the RNS limbs of the BFV ciphertext ring.
//
// Every prime p used on the GPU lies in (2^53, 2^54) and satisfies
// p = 1 mod 2N (negacyclic NTT-friendly); t = 65537 is handled separately.
// Residues are kept as uint64 in [0, p) at kernel boundaries and lazily in
// [0, 4p) inside the NTT butterflies (4p < 2^56).
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
PEPSI_HD uint64_t shoup(uint64_t x, uint64_t w, uint64_t wq, uint64_t p) {
  uint64_t r = shoup_lazy(x, w, wq, p);
  return r >= p ? r - p : r;
}
PEPSI_HD uint64_t shoup_companion(uint64_t w, uint64_t p) {
  return (uint64_t)(((u128)w << 64) / p);
}

// x mod p for x = hi:lo < 2^116 (Barrett with the quotient estimated from
// x >> 52; the estimate is at most 2 short, so two corrections suffice).
PEPSI_HD uint64_t reduce116(uint64_t lo, uint64_t hi, const Prime& P) {
  uint64_t top = (lo >> 52) | (hi << 12);          // floor(x / 2^52) < 2^64
  uint64_t q = mulhi64(top, P.barrett);            // ~ floor(x / p)
  uint64_t r = lo - q * P.p;                       // true remainder + k p, k in {0,1,2}
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
