/*
 * Oracle (test infrastructure only): a small fixed-width big integer.
 *
 * Two's complement, little-endian 64-bit words, BN_WORDS words (1280 bits),
 * enough for every exact integer the textbook FV product needs at N <= 2^14
 * and Q <= 2^440 (tensor coefficients stay below N * Q^2 / 2, times t).
 * Division is plain binary long division.
 */
#include "bignum.h"
#include <string.h>

void bn_zero(bn* r) { memset(r->w, 0, sizeof(r->w)); }
void bn_set_u64(bn* r, uint64_t v) { bn_zero(r); r->w[0] = v; }
void bn_set_i64(bn* r, int64_t v) {
  uint64_t fill = v < 0 ? ~(uint64_t)0 : 0;
  for (int i = 0; i < BN_WORDS; i++) r->w[i] = fill;
  r->w[0] = (uint64_t)v;
}
int bn_is_neg(const bn* a) { return (int)(a->w[BN_WORDS - 1] >> 63); }
int bn_is_zero(const bn* a) {
  for (int i = 0; i < BN_WORDS; i++) if (a->w[i]) return 0;
  return 1;
}
void bn_add(bn* r, const bn* a, const bn* b) {
  u128 c = 0;
  for (int i = 0; i < BN_WORDS; i++) {
    c += (u128)a->w[i] + b->w[i];
    r->w[i] = (uint64_t)c;
    c >>= 64;
  }
}
void bn_sub(bn* r, const bn* a, const bn* b) {
  uint64_t borrow = 0;
  for (int i = 0; i < BN_WORDS; i++) {
    u128 d = (u128)a->w[i] - b->w[i] - borrow;
    r->w[i] = (uint64_t)d;
    borrow = (uint64_t)(d >> 64) & 1;
  }
}
void bn_neg(bn* r, const bn* a) {
  bn z; bn_zero(&z); bn_sub(r, &z, a);
}
void bn_abs(bn* r, const bn* a) {
  if (bn_is_neg(a)) bn_neg(r, a); else *r = *a;
}
/* r = a * v mod 2^(64*BN_WORDS); correct for signed a as long as it fits. */
void bn_mul_u64(bn* r, const bn* a, uint64_t v) {
  u128 c = 0;
  bn out;
  for (int i = 0; i < BN_WORDS; i++) {
    c += (u128)a->w[i] * v;
    out.w[i] = (uint64_t)c;
    c >>= 64;
  }
  *r = out;
}
/* r = a * b mod 2^(64*BN_WORDS) (schoolbook); signed-correct when it fits. */
void bn_mul(bn* r, const bn* a, const bn* b) {
  bn out; bn_zero(&out);
  for (int i = 0; i < BN_WORDS; i++) {
    if (a->w[i] == 0) continue;
    u128 c = 0;
    for (int j = 0; i + j < BN_WORDS; j++) {
      c += (u128)a->w[i] * b->w[j] + out.w[i + j];
      out.w[i + j] = (uint64_t)c;
      c >>= 64;
    }
  }
  *r = out;
}
/* unsigned comparison */
int bn_cmp(const bn* a, const bn* b) {
  for (int i = BN_WORDS - 1; i >= 0; i--) {
    if (a->w[i] != b->w[i]) return a->w[i] < b->w[i] ? -1 : 1;
  }
  return 0;
}
/* signed comparison */
int bn_scmp(const bn* a, const bn* b) {
  int na = bn_is_neg(a), nb = bn_is_neg(b);
  if (na != nb) return na ? -1 : 1;
  return bn_cmp(a, b);
}
void bn_shl1(bn* r, const bn* a) {
  uint64_t carry = 0;
  for (int i = 0; i < BN_WORDS; i++) {
    uint64_t w = a->w[i];
    r->w[i] = (w << 1) | carry;
    carry = w >> 63;
  }
}
int bn_bitlen(const bn* a) {  /* a >= 0 */
  for (int i = BN_WORDS - 1; i >= 0; i--)
    if (a->w[i]) return 64 * i + (64 - __builtin_clzll(a->w[i]));
  return 0;
}
int bn_bit(const bn* a, int k) { return (int)((a->w[k / 64] >> (k % 64)) & 1); }
/* quotient and remainder of a / d for a >= 0, d > 0 (binary long division) */
void bn_udivmod(bn* quot, bn* rem, const bn* a, const bn* d) {
  bn q, r;
  bn_zero(&q); bn_zero(&r);
  for (int k = bn_bitlen(a) - 1; k >= 0; k--) {
    bn_shl1(&r, &r);
    r.w[0] |= (uint64_t)bn_bit(a, k);
    if (bn_cmp(&r, d) >= 0) {
      bn_sub(&r, &r, d);
      q.w[k / 64] |= (uint64_t)1 << (k % 64);
    }
  }
  if (quot) *quot = q;
  if (rem) *rem = r;
}
/* a mod m for a >= 0 (Horner over the words) */
uint64_t bn_mod_u64(const bn* a, uint64_t m) {
  u128 r = 0;
  for (int i = BN_WORDS - 1; i >= 0; i--) r = ((r << 64) | a->w[i]) % m;
  return (uint64_t)r;
}
/* a mod m into [0, m) for any signed a */
uint64_t bn_smod_u64(const bn* a, uint64_t m) {
  if (!bn_is_neg(a)) return bn_mod_u64(a, m);
  bn p; bn_neg(&p, a);
  uint64_t v = bn_mod_u64(&p, m);
  return v == 0 ? 0 : m - v;
}
