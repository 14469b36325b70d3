/*
 * Oracle (test infrastructure only): word-size modular arithmetic and
 * negacyclic polynomial products in Z_m[X]/(X^n + 1).
 *
 * Every operation is written in its plainest form: the product of two
 * residues is taken as an exact 128-bit integer and reduced with '%'.
 */
#include "oracle.h"
#include <stdlib.h>
#include <string.h>

uint64_t or_mulmod(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)(((u128)a * b) % m);
}
uint64_t or_addmod(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)(((u128)a + b) % m);
}
uint64_t or_submod(uint64_t a, uint64_t b, uint64_t m) {
  return (uint64_t)(((u128)a + m - (b % m)) % m);
}
uint64_t or_powmod(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  while (e) {
    if (e & 1) r = or_mulmod(r, a, m);
    a = or_mulmod(a, a, m);
    e >>= 1;
  }
  return r;
}
/* Fermat: a^(m-2) for prime m. */
uint64_t or_invmod(uint64_t a, uint64_t m) { return or_powmod(a, m - 2, m); }

/* Schoolbook negacyclic product: X^n = -1, so a term a_i b_j with i+j >= n
 * lands on X^(i+j-n) with a minus sign. */
void or_poly_mul_schoolbook(const uint64_t* a, const uint64_t* b, uint64_t* c,
                            int n, uint64_t m) {
  for (int k = 0; k < n; k++) c[k] = 0;
  for (int i = 0; i < n; i++) {
    if (a[i] == 0) continue;
    for (int j = 0; j < n; j++) {
      uint64_t p = or_mulmod(a[i], b[j], m);
      int k = i + j;
      if (k < n) c[k] = or_addmod(c[k], p, m);
      else c[k - n] = or_submod(c[k - n], p, m);
    }
  }
}

uint64_t or_poly_eval_point(const uint64_t* a, int n, uint64_t m, uint64_t x) {
  uint64_t r = 0;
  for (int i = n - 1; i >= 0; i--) r = or_addmod(or_mulmod(r, x, m), a[i], m);
  return r;
}

/* Evaluation at the roots x_k = psi^(2k+1), k in [n], of X^n + 1.
 * Split a(x) = a_e(x^2) + x * a_o(x^2).  The squares x_k^2 = (psi^2)^(2k+1)
 * are the roots of X^(n/2) + 1 for the primitive n-th root psi^2, and
 * x_{k+n/2}^2 = x_k^2, so
 *   A[k]       = E(a_e)[k] + x_k * E(a_o)[k]
 *   A[k + n/2] = E(a_e)[k] - x_k * E(a_o)[k]     (x_{k+n/2} = -x_k).
 * 'ws' is scratch of at least 4n words (2n for this level, the rest below). */
static void eval_rec(const uint64_t* a, uint64_t* out, int n, uint64_t m,
                     uint64_t psi, uint64_t* ws) {
  if (n == 1) { out[0] = a[0] % m; return; }
  int h = n / 2;
  uint64_t *ae = ws, *ao = ws + h, *Ee = ws + 2 * h, *Eo = ws + 3 * h;
  for (int i = 0; i < h; i++) { ae[i] = a[2 * i]; ao[i] = a[2 * i + 1]; }
  uint64_t psi2 = or_mulmod(psi, psi, m);
  eval_rec(ae, Ee, h, m, psi2, ws + 4 * h);
  eval_rec(ao, Eo, h, m, psi2, ws + 4 * h);
  uint64_t x = psi;                 /* x_0 = psi^1 */
  for (int k = 0; k < h; k++) {
    uint64_t t = or_mulmod(x, Eo[k], m);
    out[k] = or_addmod(Ee[k], t, m);
    out[k + h] = or_submod(Ee[k], t, m);
    x = or_mulmod(x, psi2, m);      /* x_{k+1} = x_k * psi^2 */
  }
}

void or_eval_fwd(uint64_t* a, int n, uint64_t m, uint64_t psi) {
  uint64_t* ws = (uint64_t*)malloc(sizeof(uint64_t) * (5 * (size_t)n + 4));
  uint64_t* out = ws + 4 * (size_t)n + 4;
  eval_rec(a, out, n, m, psi, ws);
  memcpy(a, out, sizeof(uint64_t) * n);
  free(ws);
}

/* Interpolation, undoing eval_rec step by step:
 *   E(a_e)[k] = (A[k] + A[k+n/2]) / 2,  E(a_o)[k] = (A[k] - A[k+n/2]) / (2 x_k).
 * psi_inv = psi^-1 and inv2 = 2^-1 are passed down with the recursion. */
static void interp_rec(const uint64_t* A, uint64_t* a, int n, uint64_t m,
                       uint64_t psi_inv, uint64_t inv2, uint64_t* ws) {
  if (n == 1) { a[0] = A[0] % m; return; }
  int h = n / 2;
  uint64_t *Ee = ws, *Eo = ws + h, *ae = ws + 2 * h, *ao = ws + 3 * h;
  uint64_t psi2_inv = or_mulmod(psi_inv, psi_inv, m);
  uint64_t x_inv = psi_inv;         /* x_k^-1 = psi^-(2k+1) */
  for (int k = 0; k < h; k++) {
    Ee[k] = or_mulmod(or_addmod(A[k], A[k + h], m), inv2, m);
    uint64_t d = or_mulmod(or_submod(A[k], A[k + h], m), inv2, m);
    Eo[k] = or_mulmod(d, x_inv, m);
    x_inv = or_mulmod(x_inv, psi2_inv, m);
  }
  interp_rec(Ee, ae, h, m, psi2_inv, inv2, ws + 4 * h);
  interp_rec(Eo, ao, h, m, psi2_inv, inv2, ws + 4 * h);
  for (int i = 0; i < h; i++) { a[2 * i] = ae[i]; a[2 * i + 1] = ao[i]; }
}

void or_eval_inv(uint64_t* a, int n, uint64_t m, uint64_t psi) {
  uint64_t* ws = (uint64_t*)malloc(sizeof(uint64_t) * (5 * (size_t)n + 4));
  uint64_t* out = ws + 4 * (size_t)n + 4;
  interp_rec(a, out, n, m, or_invmod(psi, m), or_invmod(2 % m, m), ws);
  memcpy(a, out, sizeof(uint64_t) * n);
  free(ws);
}

void or_poly_mul_eval(const uint64_t* a, const uint64_t* b, uint64_t* c,
                      int n, uint64_t m, uint64_t psi) {
  uint64_t* A = (uint64_t*)malloc(sizeof(uint64_t) * n);
  uint64_t* B = (uint64_t*)malloc(sizeof(uint64_t) * n);
  memcpy(A, a, sizeof(uint64_t) * n);
  memcpy(B, b, sizeof(uint64_t) * n);
  or_eval_fwd(A, n, m, psi);
  or_eval_fwd(B, n, m, psi);
  for (int k = 0; k < n; k++) c[k] = or_mulmod(A[k], B[k], m);
  or_eval_inv(c, n, m, psi);
  free(A); free(B);
}
