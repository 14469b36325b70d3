/*
 * Oracle (test infrastructure only): textbook FV (Fan-Vercauteren) over the
 * RNS representation of Q, following the operation list of the paper's
 * Sec. 3.1 (addition, plaintext multiplication, ciphertext multiplication),
 * the batching of Sec. 4.1 and the secret-key encryption of Alg. 6.
 *
 * Polynomial products modulo one prime use the evaluation map at the roots
 * of X^N + 1 (or_poly_mul_eval); the exact ciphertext product works on the
 * centred integer lifts with the big integers of bignum.c.
 */
#include "ctx.h"
#include <stdlib.h>
#include <string.h>

or_ctx* or_ctx_create(int n, int L, const uint64_t* primes, const uint64_t* psis,
                      uint64_t t, uint64_t psi_t) {
  if (L < 1 || L > OR_MAXL) return NULL;
  or_ctx* c = (or_ctx*)calloc(1, sizeof(or_ctx));
  c->n = n; c->L = L; c->t = t; c->psi_t = psi_t;
  bn_set_u64(&c->Q, 1);
  for (int i = 0; i < L; i++) {
    c->q[i] = primes[i];
    c->psi[i] = psis[i];
    bn_mul_u64(&c->Q, &c->Q, primes[i]);
  }
  for (int i = 0; i < L; i++) {
    bn_set_u64(&c->Qi[i], 1);
    for (int j = 0; j < L; j++)
      if (j != i) bn_mul_u64(&c->Qi[i], &c->Qi[i], primes[j]);
    c->Qi_mod[i] = bn_mod_u64(&c->Qi[i], primes[i]);
    c->Qi_inv[i] = or_invmod(c->Qi_mod[i], primes[i]);
  }
  bn tb; bn_set_u64(&tb, t);
  bn_udivmod(&c->Delta, NULL, &c->Q, &tb);
  for (int i = 0; i < L; i++) c->delta[i] = bn_mod_u64(&c->Delta, primes[i]);
  c->q_bits = bn_bitlen(&c->Q);
  return c;
}
void or_ctx_destroy(or_ctx* c) { free(c); }

void or_ctx_delta(const or_ctx* c, uint64_t* delta_res, int* q_bits, uint64_t* q_mod_t) {
  if (delta_res) for (int i = 0; i < c->L; i++) delta_res[i] = c->delta[i];
  if (q_bits) *q_bits = c->q_bits;
  if (q_mod_t) *q_mod_t = bn_mod_u64(&c->Q, c->t);
}

/* ---------- helpers ---------- */

/* The integer x in [0, Q) with x = res[l] mod q_l (CRT):
 *   x = sum_l [res_l * (Q/q_l)^-1]_{q_l} * (Q/q_l)  mod Q. */
static void crt(const or_ctx* c, const uint64_t* res, bn* x) {
  bn acc, term; bn_zero(&acc);
  for (int l = 0; l < c->L; l++) {
    uint64_t y = or_mulmod(res[l], c->Qi_inv[l], c->q[l]);
    bn_mul_u64(&term, &c->Qi[l], y);
    bn_add(&acc, &acc, &term);
  }
  while (bn_cmp(&acc, &c->Q) >= 0) bn_sub(&acc, &acc, &c->Q);
  *x = acc;
}
/* centred lift [x]_Q in (-Q/2, Q/2] (Q is odd, so 2x > Q decides) */
static void crt_centred(const or_ctx* c, const uint64_t* res, bn* x) {
  crt(c, res, x);
  bn twice; bn_shl1(&twice, x);
  if (bn_cmp(&twice, &c->Q) > 0) bn_sub(x, x, &c->Q);
}
void or_crt_centred(const or_ctx* c, const uint64_t* res, bn* x) { crt_centred(c, res, x); }

/* gather the L residues of coefficient i of a limb-major polynomial */
static void gather(const or_ctx* c, const uint64_t* poly, int i, uint64_t* res) {
  for (int l = 0; l < c->L; l++) res[l] = poly[(size_t)l * c->n + i];
}
/* product of two polynomials mod q_l */
static void mul_limb(const or_ctx* c, int l, const uint64_t* a, const uint64_t* b, uint64_t* out) {
  or_poly_mul_eval(a, b, out, c->n, c->q[l], c->psi[l]);
}

/* ---------- batching ---------- */

void or_encode(const or_ctx* c, const uint32_t* slots, uint32_t* poly) {
  uint64_t* a = (uint64_t*)malloc(sizeof(uint64_t) * c->n);
  for (int k = 0; k < c->n; k++) a[k] = slots[k] % c->t;
  or_eval_inv(a, c->n, c->t, c->psi_t);
  for (int k = 0; k < c->n; k++) poly[k] = (uint32_t)a[k];
  free(a);
}
void or_decode(const or_ctx* c, const uint32_t* poly, uint32_t* slots) {
  uint64_t* a = (uint64_t*)malloc(sizeof(uint64_t) * c->n);
  for (int k = 0; k < c->n; k++) a[k] = poly[k] % c->t;
  or_eval_fwd(a, c->n, c->t, c->psi_t);
  for (int k = 0; k < c->n; k++) slots[k] = (uint32_t)a[k];
  free(a);
}

/* ---------- encryption / decryption ---------- */

void or_encrypt(const or_ctx* c, const int8_t* sk, const uint32_t* m_poly,
                const uint64_t* a, const int32_t* e, uint64_t* ct) {
  int n = c->n, L = c->L;
  uint64_t* s = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* as = (uint64_t*)malloc(sizeof(uint64_t) * n);
  for (int l = 0; l < L; l++) {
    uint64_t q = c->q[l];
    for (int i = 0; i < n; i++) s[i] = smod(sk[i], q);
    mul_limb(c, l, a + (size_t)l * n, s, as);
    uint64_t* c0 = ct + (size_t)l * n;
    uint64_t* c1 = ct + (size_t)(L + l) * n;
    for (int i = 0; i < n; i++) {
      uint64_t v = or_addmod(as[i], smod(e[i], q), q);            /* a*s + e */
      uint64_t dm = or_mulmod(c->delta[l], smod(centre_t(m_poly[i], c->t), q), q);
      c0[i] = or_submod(dm, v, q);                                /* Delta*[m]_t - (a*s+e) */
      c1[i] = a[(size_t)l * n + i];
    }
  }
  free(s); free(as);
}

/* x = c0 + c1*s mod Q, limb-major */
static void phase(const or_ctx* c, const int8_t* sk, const uint64_t* ct, uint64_t* x) {
  int n = c->n, L = c->L;
  uint64_t* s = (uint64_t*)malloc(sizeof(uint64_t) * n);
  for (int l = 0; l < L; l++) {
    uint64_t q = c->q[l];
    for (int i = 0; i < n; i++) s[i] = smod(sk[i], q);
    mul_limb(c, l, ct + (size_t)(L + l) * n, s, x + (size_t)l * n);
    for (int i = 0; i < n; i++)
      x[(size_t)l * n + i] = or_addmod(x[(size_t)l * n + i], ct[(size_t)l * n + i], q);
  }
  free(s);
}

void or_decrypt_poly(const or_ctx* c, const int8_t* sk, const uint64_t* ct, uint32_t* m_poly) {
  int n = c->n, L = c->L;
  uint64_t* x = (uint64_t*)malloc(sizeof(uint64_t) * n * L);
  phase(c, sk, ct, x);
  bn twoQ; bn_shl1(&twoQ, &c->Q);
  for (int i = 0; i < n; i++) {
    uint64_t res[OR_MAXL];
    bn v, num, quot;
    gather(c, x, i, res);
    crt(c, res, &v);                      /* v in [0, Q) */
    bn_mul_u64(&num, &v, 2 * c->t);       /* 2 t v + Q, then floor-divide by 2Q */
    bn_add(&num, &num, &c->Q);
    bn_udivmod(&quot, NULL, &num, &twoQ);  /* = round(t v / Q) */
    m_poly[i] = (uint32_t)bn_mod_u64(&quot, c->t);
  }
  free(x);
}

int or_noise_budget(const or_ctx* c, const int8_t* sk, const uint64_t* ct) {
  int n = c->n, L = c->L;
  uint64_t* x = (uint64_t*)malloc(sizeof(uint64_t) * n * L);
  phase(c, sk, ct, x);
  int worst = 0;
  for (int i = 0; i < n; i++) {
    uint64_t res[OR_MAXL];
    for (int l = 0; l < L; l++)
      res[l] = or_mulmod(x[(size_t)l * n + i], c->t % c->q[l], c->q[l]);   /* t*x */
    bn v, av;
    crt_centred(c, res, &v);
    bn_abs(&av, &v);
    int b = bn_bitlen(&av);
    if (b > worst) worst = b;
  }
  free(x);
  return c->q_bits - worst - 1;
}

/* ---------- keys ---------- */

void or_keygen_relin(const or_ctx* c, const int8_t* sk, const uint64_t* a,
                     const int32_t* e, uint64_t* rlk) {
  int n = c->n, L = c->L;
  uint64_t* s = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* s2 = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* as = (uint64_t*)malloc(sizeof(uint64_t) * n);
  for (int i = 0; i < L; i++) {              /* key index (gadget digit) */
    for (int l = 0; l < L; l++) {            /* limb */
      uint64_t q = c->q[l];
      for (int k = 0; k < n; k++) s[k] = smod(sk[k], q);
      mul_limb(c, l, s, s, s2);                                      /* s^2 */
      const uint64_t* ai = a + ((size_t)i * L + l) * n;
      mul_limb(c, l, ai, s, as);
      uint64_t g = bn_mod_u64(&c->Qi[i], q);                         /* (Q/q_i) mod q_l */
      uint64_t* r0 = rlk + (((size_t)i * 2 + 0) * L + l) * n;
      uint64_t* r1 = rlk + (((size_t)i * 2 + 1) * L + l) * n;
      for (int k = 0; k < n; k++) {
        uint64_t v = or_addmod(as[k], smod(e[(size_t)i * n + k], q), q);
        r0[k] = or_submod(or_mulmod(g, s2[k], q), v, q);
        r1[k] = ai[k];
      }
    }
  }
  free(s); free(s2); free(as);
}

/* ---------- homomorphic operations ---------- */

void or_mul_plain(const or_ctx* c, const uint64_t* ct, const uint32_t* p_poly, uint64_t* out) {
  int n = c->n, L = c->L;
  uint64_t* p = (uint64_t*)malloc(sizeof(uint64_t) * n);
  for (int l = 0; l < L; l++) {
    uint64_t q = c->q[l];
    for (int i = 0; i < n; i++) p[i] = smod(centre_t(p_poly[i], c->t), q);
    for (int comp = 0; comp < 2; comp++)
      mul_limb(c, l, ct + (size_t)(comp * L + l) * n, p, out + (size_t)(comp * L + l) * n);
  }
  free(p);
}

void or_add_plain_const(const or_ctx* c, uint64_t* ct, uint32_t kappa) {
  int64_t kc = centre_t(kappa % c->t, c->t);
  for (int l = 0; l < c->L; l++) {
    uint64_t q = c->q[l];
    uint64_t v = or_mulmod(c->delta[l], smod(kc, q), q);
    ct[(size_t)l * c->n + 0] = or_addmod(ct[(size_t)l * c->n + 0], v, q);
  }
}

void or_add_plain(const or_ctx* c, uint64_t* ct, const uint32_t* p_poly) {
  for (int l = 0; l < c->L; l++) {
    uint64_t q = c->q[l];
    for (int i = 0; i < c->n; i++) {
      uint64_t v = or_mulmod(c->delta[l], smod(centre_t(p_poly[i], c->t), q), q);
      ct[(size_t)l * c->n + i] = or_addmod(ct[(size_t)l * c->n + i], v, q);
    }
  }
}

void or_mul_const(const or_ctx* c, uint64_t* ct, uint32_t k) {
  int64_t kc = centre_t(k % c->t, c->t);
  for (int l = 0; l < c->L; l++) {
    uint64_t q = c->q[l], kq = smod(kc, q);
    for (int comp = 0; comp < 2; comp++)
      for (int i = 0; i < c->n; i++) {
        uint64_t* v = ct + (size_t)(comp * c->L + l) * c->n + i;
        *v = or_mulmod(*v, kq, q);
      }
  }
}

/* acc (aw words, two's complement) += sign * (x * y), x, y magnitudes of lw words */
static void acc_addmul(uint64_t* acc, int aw, const uint64_t* x, const uint64_t* y,
                       int lw, int negative) {
  uint64_t p[2 * OR_MAXL + 2];
  memset(p, 0, sizeof(uint64_t) * 2 * lw);
  for (int i = 0; i < lw; i++) {
    u128 carry = 0;
    for (int j = 0; j < lw; j++) {
      carry += (u128)x[i] * y[j] + p[i + j];
      p[i + j] = (uint64_t)carry;
      carry >>= 64;
    }
    p[i + lw] = (uint64_t)carry;
  }
  if (!negative) {
    u128 c = 0;
    for (int i = 0; i < aw; i++) {
      c += (u128)acc[i] + (i < 2 * lw ? p[i] : 0);
      acc[i] = (uint64_t)c;
      c >>= 64;
    }
  } else {
    uint64_t borrow = 0;
    for (int i = 0; i < aw; i++) {
      u128 d = (u128)acc[i] - (i < 2 * lw ? p[i] : 0) - borrow;
      acc[i] = (uint64_t)d;
      borrow = (uint64_t)(d >> 64) & 1;
    }
  }
}

/* sign/magnitude form of a centred lift */
typedef struct { int neg; uint64_t mag[OR_MAXL + 1]; } lifted;

static void lift_poly(const or_ctx* c, const uint64_t* poly, lifted* out) {
  for (int i = 0; i < c->n; i++) {
    uint64_t res[OR_MAXL];
    bn x, ax;
    gather(c, poly, i, res);
    crt_centred(c, res, &x);
    out[i].neg = bn_is_neg(&x);
    bn_abs(&ax, &x);
    for (int w = 0; w <= c->L; w++) out[i].mag[w] = ax.w[w];
  }
}

/* FV multiplication: d = x (x) y over Z[X]/(X^N+1) on centred lifts,
 *   d0 = x0*y0,  d1 = x0*y1 + x1*y0,  d2 = x1*y1,
 * then out_k = [round(t * d_k / Q)]_Q. */
void or_multiply(const or_ctx* c, const uint64_t* x, const uint64_t* y, uint64_t* out3) {
  int n = c->n, L = c->L;
  int lw = L;                     /* words of a lifted magnitude (|v| < Q/2 < 2^(64L)) */
  int aw = 2 * lw + 1;            /* accumulator words */
  lifted* X0 = (lifted*)malloc(sizeof(lifted) * n);
  lifted* X1 = (lifted*)malloc(sizeof(lifted) * n);
  lifted* Y0 = (lifted*)malloc(sizeof(lifted) * n);
  lifted* Y1 = (lifted*)malloc(sizeof(lifted) * n);
  lift_poly(c, x, X0);
  lift_poly(c, x + (size_t)L * n, X1);
  lift_poly(c, y, Y0);
  lift_poly(c, y + (size_t)L * n, Y1);
  bn twoQ; bn_shl1(&twoQ, &c->Q);
#pragma omp parallel for schedule(dynamic, 16)
  for (int k = 0; k < n; k++) {
    uint64_t acc[3][2 * OR_MAXL + 4];
    memset(acc, 0, sizeof(acc));
    /* coefficient k collects a_i b_j with i + j = k (sign +) or i + j = k + n (sign -) */
    for (int i = 0; i < n; i++) {
      int j = k - i, neg = 0;
      if (j < 0) { j += n; neg = 1; }
      acc_addmul(acc[0], aw, X0[i].mag, Y0[j].mag, lw, neg ^ X0[i].neg ^ Y0[j].neg);
      acc_addmul(acc[1], aw, X0[i].mag, Y1[j].mag, lw, neg ^ X0[i].neg ^ Y1[j].neg);
      acc_addmul(acc[1], aw, X1[i].mag, Y0[j].mag, lw, neg ^ X1[i].neg ^ Y0[j].neg);
      acc_addmul(acc[2], aw, X1[i].mag, Y1[j].mag, lw, neg ^ X1[i].neg ^ Y1[j].neg);
    }
    for (int comp = 0; comp < 3; comp++) {
      bn d, num, quot, r;
      /* sign-extend the accumulator into a bn */
      uint64_t fill = (acc[comp][aw - 1] >> 63) ? ~(uint64_t)0 : 0;
      for (int w = 0; w < BN_WORDS; w++) d.w[w] = w < aw ? acc[comp][w] : fill;
      int neg = bn_is_neg(&d);
      bn_abs(&d, &d);
      /* round(t |d| / Q) = floor((2 t |d| + Q) / 2Q); ties cannot occur (Q odd, gcd(t,Q)=1) */
      bn_mul_u64(&num, &d, 2 * c->t);
      bn_add(&num, &num, &c->Q);
      bn_udivmod(&quot, NULL, &num, &twoQ);
      if (neg) bn_neg(&r, &quot); else r = quot;
      for (int l = 0; l < L; l++)
        out3[((size_t)comp * L + l) * n + k] = bn_smod_u64(&r, c->q[l]);
    }
  }
  free(X0); free(X1); free(Y0); free(Y1);
}

/* Relinearisation with the RNS gadget: digits D_i = [d2 * (Q/q_i)^-1]_{q_i} in [0, q_i),
 * so that sum_i D_i (Q/q_i) = d2 mod Q;  out = (d0 + sum_i D_i rlk_i0, d1 + sum_i D_i rlk_i1). */
void or_relin(const or_ctx* c, const uint64_t* ct3, const uint64_t* rlk, uint64_t* out) {
  int n = c->n, L = c->L;
  uint64_t* D = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* Dj = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* prod = (uint64_t*)malloc(sizeof(uint64_t) * n);
  memcpy(out, ct3, sizeof(uint64_t) * 2 * L * n);         /* d0, d1 */
  for (int i = 0; i < L; i++) {
    const uint64_t* d2i = ct3 + (size_t)(2 * L + i) * n;
    for (int k = 0; k < n; k++) D[k] = or_mulmod(d2i[k], c->Qi_inv[i], c->q[i]);
    for (int l = 0; l < L; l++) {
      uint64_t q = c->q[l];
      for (int k = 0; k < n; k++) Dj[k] = D[k] % q;
      for (int comp = 0; comp < 2; comp++) {
        const uint64_t* r = rlk + (((size_t)i * 2 + comp) * L + l) * n;
        mul_limb(c, l, Dj, r, prod);
        uint64_t* o = out + (size_t)(comp * L + l) * n;
        for (int k = 0; k < n; k++) o[k] = or_addmod(o[k], prod[k], q);
      }
    }
  }
  free(D); free(Dj); free(prod);
}

/* ---------- many at once (independent, so spread over threads) ---------- */

void or_encode_many(const or_ctx* c, const uint32_t* slots, int count, uint32_t* polys) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int i = 0; i < count; i++)
    or_encode(c, slots + (size_t)i * c->n, polys + (size_t)i * c->n);
}

void or_encrypt_many(const or_ctx* c, const int8_t* sk, const uint32_t* m_polys, const uint64_t* a,
                     const int32_t* e, int count, uint64_t* ct) {
#pragma omp parallel for schedule(dynamic, 2)
  for (int i = 0; i < count; i++)
    or_encrypt(c, sk, m_polys + (size_t)i * c->n, a + (size_t)i * c->L * c->n,
               e + (size_t)i * c->n, ct + (size_t)i * 2 * c->L * c->n);
}
