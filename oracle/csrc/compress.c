/*
 * Oracle (test infrastructure only): request and response compression.
 *
 * Request: the c1 part of a secret-key ciphertext is the uniform polynomial a; it can be sent
 * as a 32-byte seed and expanded by the receiver.  Reading (the paper only reports the
 * compressed sizes, Table "dipsi-cpsi"): ChaCha20 of RFC 8439 (20 rounds, 32-bit words,
 * little-endian), key = the seed, nonce = (j, l, 0) for ciphertext j and limb l, block counter
 * b from 0; coefficient k takes the 16 keystream bytes [16k, 16k + 16) of that stream as a
 * little-endian 128-bit integer W, and a_{j,l}[k] = W mod q_l (the bias of W mod q is below
 * q / 2^128 < 2^-74).
 *
 * Response: modulus switching to the first prime, c' = [round(q_0 c / Q)]_{q_0} on the centred
 * lift of each coefficient, written out with exact integers.
 */
#include "ctx.h"
#include "bignum.h"
#include <stdlib.h>
#include <string.h>

static uint32_t rotl(uint32_t x, int r) { return (x << r) | (x >> (32 - r)); }

void or_chacha_quarter(uint32_t* a, uint32_t* b, uint32_t* c, uint32_t* d) {
  *a += *b; *d ^= *a; *d = rotl(*d, 16);
  *c += *d; *b ^= *c; *b = rotl(*b, 12);
  *a += *b; *d ^= *a; *d = rotl(*d, 8);
  *c += *d; *b ^= *c; *b = rotl(*b, 7);
}

/* RFC 8439 Sec. 2.3: state = constants | key | counter | nonce; 10 double rounds (column,
 * then diagonal quarter rounds); output = state after the rounds + the initial state. */
void or_chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3], uint32_t out[16]) {
  uint32_t s[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u};
  for (int i = 0; i < 8; i++) s[4 + i] = key[i];
  s[12] = counter;
  for (int i = 0; i < 3; i++) s[13 + i] = nonce[i];
  uint32_t x[16];
  memcpy(x, s, sizeof(x));
  for (int r = 0; r < 10; r++) {
    or_chacha_quarter(&x[0], &x[4], &x[8], &x[12]);
    or_chacha_quarter(&x[1], &x[5], &x[9], &x[13]);
    or_chacha_quarter(&x[2], &x[6], &x[10], &x[14]);
    or_chacha_quarter(&x[3], &x[7], &x[11], &x[15]);
    or_chacha_quarter(&x[0], &x[5], &x[10], &x[15]);
    or_chacha_quarter(&x[1], &x[6], &x[11], &x[12]);
    or_chacha_quarter(&x[2], &x[7], &x[8], &x[13]);
    or_chacha_quarter(&x[3], &x[4], &x[9], &x[14]);
  }
  for (int i = 0; i < 16; i++) out[i] = x[i] + s[i];
}

/* a_j for j in [first, first + count): out[(j - first) * stride + l * N + k] */
void or_expand_uniform(const or_ctx* c, const uint8_t seed[32], int first, int count, uint64_t* out,
                       size_t stride) {
  int n = c->n, L = c->L;
  uint32_t key[8];
  for (int i = 0; i < 8; i++)
    key[i] = (uint32_t)seed[4 * i] | (uint32_t)seed[4 * i + 1] << 8 | (uint32_t)seed[4 * i + 2] << 16 |
             (uint32_t)seed[4 * i + 3] << 24;
#pragma omp parallel for schedule(static) collapse(2)
  for (int jj = 0; jj < count; jj++)
    for (int l = 0; l < L; l++) {
      uint32_t nonce[3] = {(uint32_t)(first + jj), (uint32_t)l, 0};
      uint32_t blk[16];
      for (int k = 0; k < n; k++) {
        if (k % 4 == 0) or_chacha20_block(key, (uint32_t)(k / 4), nonce, blk);
        const uint32_t* w = blk + 4 * (k % 4);
        u128 W = (u128)w[0] | (u128)w[1] << 32 | (u128)w[2] << 64 | (u128)w[3] << 96;
        out[(size_t)jj * stride + (size_t)l * n + k] = (uint64_t)(W % c->q[l]);
      }
    }
}

/* c' = [round(q_0 X / Q)]_{q_0} for the centred lift X of every coefficient of ct [2][L][N];
 * out [2][N].  round(q_0 X / Q) = floor((2 q_0 |X| + Q) / 2Q) with the sign of X (ties cannot
 * occur: Q / q_0 is odd). */
void or_mod_switch(const or_ctx* c, const uint64_t* ct, uint64_t* out) {
  int n = c->n, L = c->L;
  bn twoQ;
  bn_shl1(&twoQ, &c->Q);
  uint64_t* res = (uint64_t*)malloc(sizeof(uint64_t) * L);
  for (int comp = 0; comp < 2; comp++)
    for (int k = 0; k < n; k++) {
      for (int l = 0; l < L; l++) res[l] = ct[((size_t)comp * L + l) * n + k];
      bn x, ax, num, quot, r;
      or_crt_centred(c, res, &x);
      int neg = bn_is_neg(&x);
      bn_abs(&ax, &x);
      bn_mul_u64(&num, &ax, 2 * c->q[0]);
      bn_add(&num, &num, &c->Q);
      bn_udivmod(&quot, NULL, &num, &twoQ);
      if (neg) bn_neg(&r, &quot); else r = quot;
      out[(size_t)comp * n + k] = bn_smod_u64(&r, c->q[0]);
    }
  free(res);
}
