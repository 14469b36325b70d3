/* Oracle (test infrastructure only): the scheme context shared by bfv.c and server.c. */
#ifndef PEPSI_ORACLE_CTX_H
#define PEPSI_ORACLE_CTX_H
#include "bignum.h"

#define OR_MAXL 16

struct or_ctx {
  int n, L;
  uint64_t t, psi_t;
  uint64_t q[OR_MAXL], psi[OR_MAXL];
  bn Q;                      /* product of the primes */
  bn Qi[OR_MAXL];            /* Q / q_i */
  uint64_t Qi_inv[OR_MAXL];  /* (Q / q_i)^-1 mod q_i */
  bn Delta;                  /* floor(Q / t) */
  uint64_t delta[OR_MAXL];   /* Delta mod q_i */
  uint64_t Qi_mod[OR_MAXL];  /* (Q / q_i) mod q_i */
  int q_bits;
};

/* residue in [0, m) of a signed 64-bit integer */
static inline uint64_t smod(int64_t v, uint64_t m) {
  int64_t r = v % (int64_t)m;
  return (uint64_t)(r < 0 ? r + (int64_t)m : r);
}
/* centred representative of v in [0, t): (-t/2, t/2] (t odd) */
static inline int64_t centre_t(uint64_t v, uint64_t t) {
  return v <= (t - 1) / 2 ? (int64_t)v : (int64_t)v - (int64_t)t;
}
/* centred CRT lift of one coefficient's residues (bfv.c) */
void or_crt_centred(const or_ctx* c, const uint64_t* res, bn* x);

#endif
