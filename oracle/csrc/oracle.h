/*
 * PEPSI reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, textbook CPU implementation of the server computation of
 * PEPSI PSI-cardinality (arXiv 2310.14565, Sec. 3.1 FV operations, Alg. 1
 * Arith-CW-Eq, Alg. 2 Intersect, Alg. 5 PSI-Sum with unit server values).
 * Only the test suite, the smoke entry and the CPU-baseline leg of the
 * benchmark may load it.  It shares no code with the GPU library.
 *
 * Conventions (one fixed reading of what the paper leaves open):
 *   - ring R = Z[X]/(X^N + 1); Q = q_0 * ... * q_{L-1}; t plaintext modulus;
 *   - a polynomial mod Q is stored limb-major: res[l*N + i] = coeff_i mod q_l,
 *     every residue in [0, q_l);
 *   - [x]_m denotes the centred representative in (-m/2, m/2];
 *   - Delta = floor(Q / t);
 *   - a ciphertext is (c0, c1), stored c0 limbs then c1 limbs: [2][L][N].
 */
#ifndef PEPSI_ORACLE_H
#define PEPSI_ORACLE_H
#include <stdint.h>
#include <stddef.h>

typedef unsigned __int128 u128;

/* ---- modular arithmetic on one word (all moduli < 2^63) ---- */
uint64_t or_mulmod(uint64_t a, uint64_t b, uint64_t m);
uint64_t or_addmod(uint64_t a, uint64_t b, uint64_t m);
uint64_t or_submod(uint64_t a, uint64_t b, uint64_t m);
uint64_t or_powmod(uint64_t a, uint64_t e, uint64_t m);
uint64_t or_invmod(uint64_t a, uint64_t m);      /* m prime */

/* ---- negacyclic polynomials mod one prime ---- */
/* c = a*b mod (X^n+1, m) by the schoolbook definition (c may not alias). */
void or_poly_mul_schoolbook(const uint64_t* a, const uint64_t* b, uint64_t* c,
                            int n, uint64_t m);
/* Evaluate a(x) by Horner's rule. */
uint64_t or_poly_eval_point(const uint64_t* a, int n, uint64_t m, uint64_t x);
/* In place: a[k] <- a(psi^(2k+1)) for k in [n]  (natural order), where psi is
 * a primitive 2n-th root of unity mod m; the points are the n roots of X^n+1. */
void or_eval_fwd(uint64_t* a, int n, uint64_t m, uint64_t psi);
/* Inverse of or_eval_fwd (interpolation at the same points). */
void or_eval_inv(uint64_t* a, int n, uint64_t m, uint64_t psi);
/* c = a*b mod (X^n+1, m) through evaluation at the n roots of X^n+1. */
void or_poly_mul_eval(const uint64_t* a, const uint64_t* b, uint64_t* c,
                      int n, uint64_t m, uint64_t psi);

/* ---- the scheme context ---- */
typedef struct or_ctx or_ctx;
/* primes[L] pairwise distinct, each = 1 mod 2n; psis[l] a primitive 2n-th
 * root mod primes[l]; psi_t a primitive 2n-th root mod t. */
or_ctx* or_ctx_create(int n, int L, const uint64_t* primes, const uint64_t* psis,
                      uint64_t t, uint64_t psi_t);
void or_ctx_destroy(or_ctx* c);
/* Delta mod q_l for each limb, Q's bit length, Q mod t. */
void or_ctx_delta(const or_ctx* c, uint64_t* delta_res, int* q_bits, uint64_t* q_mod_t);

/* ---- batching: slots in Z_t^n <-> plaintext polynomial in R_t ---- */
/* encode: poly p with p(psi_t^(2k+1)) = slots[k]; coefficients in [0,t). */
void or_encode(const or_ctx* c, const uint32_t* slots, uint32_t* poly);
void or_decode(const or_ctx* c, const uint32_t* poly, uint32_t* slots);

/* ---- textbook FV (all ciphertexts in coefficient form) ---- */
/* ct = ([-(a*s+e) + Delta*[m]_t]_Q, a); a: [L][N] residues, e: [N] small. */
void or_encrypt(const or_ctx* c, const int8_t* sk, const uint32_t* m_poly,
                const uint64_t* a, const int32_t* e, uint64_t* ct);
/* count independent encodings / encryptions (threads over the count) */
void or_encode_many(const or_ctx* c, const uint32_t* slots, int count, uint32_t* polys);
void or_encrypt_many(const or_ctx* c, const int8_t* sk, const uint32_t* m_polys, const uint64_t* a,
                     const int32_t* e, int count, uint64_t* ct);
/* m = [round(t/Q * [c0 + c1*s]_Q)]_t, coefficients in [0,t). */
void or_decrypt_poly(const or_ctx* c, const int8_t* sk, const uint64_t* ct, uint32_t* m_poly);
/* invariant-noise budget in bits: bitlen(Q) - bitlen(max |[t*(c0+c1*s)]_Q|) - 1 */
int or_noise_budget(const or_ctx* c, const int8_t* sk, const uint64_t* ct);
/* relinearisation key, RNS gadget: rlk_i = ([-(a_i*s + e_i) + (Q/q_i)*s^2]_Q, a_i)
 * a: [L][L][N] (key i, limb l), e: [L][N]; rlk: [L][2][L][N]. */
void or_keygen_relin(const or_ctx* c, const int8_t* sk, const uint64_t* a,
                     const int32_t* e, uint64_t* rlk);
/* plaintext multiply (c0*p, c1*p), p = centred lift of a plaintext polynomial. */
void or_mul_plain(const or_ctx* c, const uint64_t* ct, const uint32_t* p_poly, uint64_t* out);
/* c0 += Delta*[kappa]_t (constant plaintext). */
void or_add_plain_const(const or_ctx* c, uint64_t* ct, uint32_t kappa);
/* c0 += Delta*[p]_t (plaintext polynomial). */
void or_add_plain(const or_ctx* c, uint64_t* ct, const uint32_t* p_poly);
/* (k*c0, k*c1) with the centred representative [k]_t. */
void or_mul_const(const or_ctx* c, uint64_t* ct, uint32_t k);
/* textbook FV product without relinearisation: out = [round(t/Q * x (x) y)]_Q,
 * x, y lifted to centred integers; out: [3][L][N]. */
void or_multiply(const or_ctx* c, const uint64_t* x, const uint64_t* y, uint64_t* out3);
/* relinearise a 3-component ciphertext with the RNS-gadget key: out: [2][L][N]. */
void or_relin(const or_ctx* c, const uint64_t* ct3, const uint64_t* rlk, uint64_t* out);

/* ---- server computation (Alg. 1 + Alg. 2 / Alg. 5) ---- */
/* Evaluate the equality ciphertext of ONE server batch (one i').
 *   cts: client ciphertexts [ell][2][L][N] (coefficient form)
 *   cw : server codeword positions for this batch, [N][h] (uint16), 0xFFFF = none
 *        (a dummy entry has all h positions 0xFFFF, i.e. the all-zero word)
 *   out: e = prod_{r in [h]} (h' - r)  (without the 1/h! factor), [2][L][N]. */
void or_server_batch(const or_ctx* c, int ell, int h, const uint64_t* cts,
                     const uint16_t* cw, const uint64_t* rlk, uint64_t* out);
/* Same, stopping after the select-and-sum: S = sum_j ct_j (*) p_j, [2][L][N]. */
void or_select_sum(const or_ctx* c, int ell, int h, const uint64_t* cts,
                   const uint16_t* cw, uint64_t* out);
/* The full server computation over batches [i0, i1) of a [mu][N][h] table:
 *   acc = sum e_{i'}  (with vals [mu][N]: sum of encode(vals[i']) * e_{i'}, Alg. 4/5);
 *   out = [(h!)^-1]_t * acc;  if mask: c0 += Delta*[encode(mask)]_t
 * (finalize != 0 applies the factor and the mask; otherwise out = acc). */
void or_server_eval(const or_ctx* c, int ell, int h, int mu_begin, int mu_end,
                    const uint64_t* cts, const uint16_t* cw_table,
                    const uint64_t* rlk, const uint32_t* mask, const uint32_t* vals,
                    int finalize, uint64_t* out);
/* ---- request and response compression (compress.c) ---- */
/* RFC 8439 ChaCha20 quarter round and block function. */
void or_chacha_quarter(uint32_t* a, uint32_t* b, uint32_t* c, uint32_t* d);
void or_chacha20_block(const uint32_t key[8], uint32_t counter, const uint32_t nonce[3], uint32_t out[16]);
/* The uniform polynomials a_j, j in [first, first + count), expanded from a 32-byte seed:
 * a_{j,l}[k] = (16 keystream bytes of ChaCha20(seed, nonce (j, l, 0)) at 16k, LE) mod q_l;
 * out[(j - first) * stride + l * N + k]. */
void or_expand_uniform(const or_ctx* c, const uint8_t seed[32], int first, int count, uint64_t* out,
                       size_t stride);
/* Modulus switching to q_0: out[c][k] = [round(q_0 X / Q)]_{q_0}, X the centred lift of
 * coefficient k of component c of ct [2][L][N]. */
void or_mod_switch(const or_ctx* c, const uint64_t* ct, uint64_t* out);

#endif
