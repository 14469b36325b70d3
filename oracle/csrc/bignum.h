/* Oracle (test infrastructure only): fixed-width two's complement big integer. */
#ifndef PEPSI_ORACLE_BIGNUM_H
#define PEPSI_ORACLE_BIGNUM_H
#include "oracle.h"

#define BN_WORDS 20
typedef struct { uint64_t w[BN_WORDS]; } bn;

void bn_zero(bn* r);
void bn_set_u64(bn* r, uint64_t v);
void bn_set_i64(bn* r, int64_t v);
int bn_is_neg(const bn* a);
int bn_is_zero(const bn* a);
void bn_add(bn* r, const bn* a, const bn* b);
void bn_sub(bn* r, const bn* a, const bn* b);
void bn_neg(bn* r, const bn* a);
void bn_abs(bn* r, const bn* a);
void bn_mul_u64(bn* r, const bn* a, uint64_t v);
void bn_mul(bn* r, const bn* a, const bn* b);
int bn_cmp(const bn* a, const bn* b);
int bn_scmp(const bn* a, const bn* b);
void bn_shl1(bn* r, const bn* a);
int bn_bitlen(const bn* a);
int bn_bit(const bn* a, int k);
void bn_udivmod(bn* quot, bn* rem, const bn* a, const bn* d);
uint64_t bn_mod_u64(const bn* a, uint64_t m);
uint64_t bn_smod_u64(const bn* a, uint64_t m);
#endif
