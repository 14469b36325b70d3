/*
 * Oracle (test infrastructure only): the server computation of PEPSI
 * PSI-cardinality.
 *   Alg. 1 (Arith-CW-Eq):  h' = sum_j x_j y_j;  e = (1/h!) prod_{r in [h]} (h' - r)
 *   Alg. 2 (Intersect):    ct_ind = sum over server batches i' of ct_eq[i']
 *   Alg. 5 (PSI-Sum):      sum over i' of val_s[i'] * ct_eq[i'] (server values as
 *                          batch-encoded plaintexts; all ones = PSI-Cardinality), plus a
 *                          mask r with sum_k r_k = 0.
 *   Alg. 4 (labelled PSI): the same sum of val_s[i'] * ct_eq[i'], no mask.
 * With the client bits encrypted slot-wise (one ciphertext per codeword bit j)
 * and the server bits as plaintexts, h' for one server batch is the sum over
 * j of the plaintext products ct_j (*) pt_s[i'][j].  The constant (1/h!) is
 * applied once to the sum over i' (it is a linear map mod Q).
 */
#include "ctx.h"
#include <stdlib.h>
#include <string.h>


/* evaluation form of every limb of every client ciphertext */
static uint64_t* eval_cts(const or_ctx* c, int ell, const uint64_t* cts) {
  int n = c->n, L = c->L;
  size_t total = (size_t)ell * 2 * L * n;
  uint64_t* E = (uint64_t*)malloc(sizeof(uint64_t) * total);
  memcpy(E, cts, sizeof(uint64_t) * total);
#pragma omp parallel for schedule(dynamic, 4)
  for (long r = 0; r < (long)ell * 2 * L; r++) {
    int l = (int)(r % L);
    or_eval_fwd(E + (size_t)r * n, n, c->q[l], c->psi[l]);
  }
  return E;
}

/* S = sum_j ct_j (*) p_j for one server batch, where p_j is the plaintext
 * whose slot k is 1 iff j is one of the h positions of the server codeword in
 * bin k.  The plaintext products are accumulated at the evaluation points of
 * X^N + 1 (the evaluation map is a ring isomorphism, so the sum of the
 * products is the interpolation of the sum of the pointwise products). */
static void select_sum_eval(const or_ctx* c, int ell, int h, const uint64_t* E,
                            const uint16_t* cw, uint64_t* out) {
  int n = c->n, L = c->L;
  uint64_t t = c->t;
  uint32_t* y = (uint32_t*)malloc(sizeof(uint32_t) * n);
  uint32_t* p = (uint32_t*)malloc(sizeof(uint32_t) * n);
  uint64_t* P = (uint64_t*)malloc(sizeof(uint64_t) * n);
  memset(out, 0, sizeof(uint64_t) * 2 * L * n);
  for (int j = 0; j < ell; j++) {
    int any = 0;
    for (int k = 0; k < n; k++) {
      y[k] = 0;
      for (int r = 0; r < h; r++) if (cw[(size_t)k * h + r] == j) y[k] = 1;
      any |= y[k];
    }
    if (!any) continue;                 /* p_j = 0 contributes nothing */
    or_encode(c, y, p);
    for (int l = 0; l < L; l++) {
      uint64_t q = c->q[l];
      for (int k = 0; k < n; k++) P[k] = smod(centre_t(p[k], t), q);
      or_eval_fwd(P, n, q, c->psi[l]);
      for (int comp = 0; comp < 2; comp++) {
        const uint64_t* Ec = E + (((size_t)j * 2 + comp) * L + l) * n;
        uint64_t* o = out + ((size_t)comp * L + l) * n;
        for (int k = 0; k < n; k++) o[k] = or_addmod(o[k], or_mulmod(Ec[k], P[k], q), q);
      }
    }
  }
  for (int comp = 0; comp < 2; comp++)
    for (int l = 0; l < L; l++)
      or_eval_inv(out + ((size_t)comp * L + l) * n, n, c->q[l], c->psi[l]);
  free(y); free(p); free(P);
}

void or_select_sum(const or_ctx* c, int ell, int h, const uint64_t* cts,
                   const uint16_t* cw, uint64_t* out) {
  uint64_t* E = eval_cts(c, ell, cts);
  select_sum_eval(c, ell, h, E, cw, out);
  free(E);
}

/* e = prod_{r in [h]} f_r with f_r = S + Delta*[-r]_t, multiplied as a
 * balanced tree (adjacent pairs, an odd one carried up), relinearising after
 * every product. */
static void equality_product(const or_ctx* c, int h, const uint64_t* S,
                             const uint64_t* rlk, uint64_t* out) {
  int n = c->n, L = c->L;
  uint64_t t = c->t;
  size_t csz = (size_t)2 * L * n;
  uint64_t* f = (uint64_t*)malloc(sizeof(uint64_t) * csz * h);
  uint64_t* g = (uint64_t*)malloc(sizeof(uint64_t) * csz * h);
  uint64_t* t3 = (uint64_t*)malloc(sizeof(uint64_t) * 3 * L * n);
  for (int r = 0; r < h; r++) {
    memcpy(f + r * csz, S, sizeof(uint64_t) * csz);
    or_add_plain_const(c, f + r * csz, (uint32_t)((t - (uint64_t)r % t) % t));
  }
  int cnt = h;
  while (cnt > 1) {
    int m = 0;
    for (int i = 0; i + 1 < cnt; i += 2) {
      or_multiply(c, f + i * csz, f + (i + 1) * csz, t3);
      or_relin(c, t3, rlk, g + (size_t)m * csz);
      m++;
    }
    if (cnt % 2) { memcpy(g + (size_t)m * csz, f + (size_t)(cnt - 1) * csz, sizeof(uint64_t) * csz); m++; }
    uint64_t* tmp = f; f = g; g = tmp;
    cnt = m;
  }
  memcpy(out, f, sizeof(uint64_t) * csz);
  free(f); free(g); free(t3);
}

void or_server_batch(const or_ctx* c, int ell, int h, const uint64_t* cts,
                     const uint16_t* cw, const uint64_t* rlk, uint64_t* out) {
  int n = c->n, L = c->L;
  uint64_t* S = (uint64_t*)malloc(sizeof(uint64_t) * 2 * L * n);
  or_select_sum(c, ell, h, cts, cw, S);
  equality_product(c, h, S, rlk, out);
  free(S);
}

void or_server_eval(const or_ctx* c, int ell, int h, int mu_begin, int mu_end,
                    const uint64_t* cts, const uint16_t* cw_table,
                    const uint64_t* rlk, const uint32_t* mask, const uint32_t* vals,
                    int finalize, uint64_t* out) {
  int n = c->n, L = c->L;
  uint64_t t = c->t;
  size_t csz = (size_t)2 * L * n;
  uint64_t* E = eval_cts(c, ell, cts);
  memset(out, 0, sizeof(uint64_t) * csz);
  /* few batches: run them one after another so the products inside use every core */
#pragma omp parallel if (mu_end - mu_begin >= 8)
  {
    uint64_t* S = (uint64_t*)malloc(sizeof(uint64_t) * csz);
    uint64_t* e = (uint64_t*)malloc(sizeof(uint64_t) * csz);
    uint64_t* part = (uint64_t*)calloc(csz, sizeof(uint64_t));
    uint32_t* vp = vals ? (uint32_t*)malloc(sizeof(uint32_t) * n) : NULL;
#pragma omp for schedule(dynamic, 1)
    for (int ip = mu_begin; ip < mu_end; ip++) {
      select_sum_eval(c, ell, h, E, cw_table + (size_t)ip * n * h, S);
      equality_product(c, h, S, rlk, e);
      if (vals) {
        /* Alg. 4 / Alg. 5: val_s[i'] * ct_eq[i'], the server values of batch i' as a
         * batch-encoded plaintext (slot k = value of the item in bin k) */
        or_encode(c, vals + (size_t)ip * n, vp);
        or_mul_plain(c, e, vp, S);
        memcpy(e, S, sizeof(uint64_t) * csz);
      }
      for (int comp = 0; comp < 2; comp++)
        for (int l = 0; l < L; l++)
          for (int k = 0; k < n; k++) {
            size_t at = ((size_t)comp * L + l) * n + k;
            part[at] = or_addmod(part[at], e[at], c->q[l]);
          }
    }
#pragma omp critical
    for (int comp = 0; comp < 2; comp++)
      for (int l = 0; l < L; l++)
        for (int k = 0; k < n; k++) {
          size_t at = ((size_t)comp * L + l) * n + k;
          out[at] = or_addmod(out[at], part[at], c->q[l]);
        }
    free(S); free(e); free(part); free(vp);
  }
  free(E);
  if (finalize) {
    uint64_t hf = 1;
    for (int r = 2; r <= h; r++) hf = or_mulmod(hf, (uint64_t)r, t);
    or_mul_const(c, out, (uint32_t)or_invmod(hf, t));     /* (h!)^-1 mod t */
    if (mask) {
      uint32_t* mp = (uint32_t*)malloc(sizeof(uint32_t) * n);
      or_encode(c, mask, mp);
      or_add_plain(c, out, mp);
      free(mp);
    }
  }
}

/* threads an OpenMP region of the oracle uses (reported beside its timings) */
#include <omp.h>
int or_num_threads(void) { return omp_get_max_threads(); }
