// Scheme parameters and the constant tables the kernels read.
//
// Prime layout: index 0..L-1 are the ciphertext primes q_i (their product is
// Q), index L..L+K-1 the auxiliary primes b_j (product B) used only inside the
// ciphertext product, where an integer below N * Q^2 must be represented
// exactly (Q * B > 2 t N Q^2 is required; K = L + 1 leaves > 20 bits spare).
#pragma once
#include <stdint.h>
#include "modarith.hpp"

#define PEPSI_MAXL 8
#define PEPSI_MAXK 9
#define PEPSI_MAXP (PEPSI_MAXL + PEPSI_MAXK)
#define PEPSI_MW 10          // 64-bit words of the multiword constants (>= 9 * 54 bits + spare)

struct MWord { uint64_t w[PEPSI_MW]; };

// A fixed-point constant c in [0, 1) * 2^k stored as floor(c * 2^128) (two words).
struct Fix128 { uint64_t lo, hi; };

struct Consts {
  int n, logn, L, K;
  Prime prm[PEPSI_MAXP];
  uint64_t n_inv[PEPSI_MAXP], n_inv_shoup[PEPSI_MAXP];
  uint32_t n_inv_t;
  uint64_t delta[PEPSI_MAXL];                 // floor(Q / t) mod q_i

  // Q -> B extension of the centred lift
  uint64_t qhat_inv[PEPSI_MAXL], qhat_inv_shoup[PEPSI_MAXL];   // (Q/q_i)^-1 mod q_i
  uint64_t qhat_mod_q[PEPSI_MAXL];            // (Q/q_i) mod q_i
  double inv_q_d[PEPSI_MAXL];                 // 1 / q_i in double precision
  uint64_t qhat_mod_b[PEPSI_MAXL][PEPSI_MAXK];// (Q/q_i) mod b_j
  uint64_t q_mod_b[PEPSI_MAXK];               // Q mod b_j

  // B -> Q extension of the centred lift
  uint64_t bhat_inv[PEPSI_MAXK], bhat_inv_shoup[PEPSI_MAXK];   // (B/b_j)^-1 mod b_j
  double inv_b_d[PEPSI_MAXK];                 // 1 / b_j in double precision
  uint64_t bhat_mod_q[PEPSI_MAXK][PEPSI_MAXL];// (B/b_j) mod q_i
  uint64_t b_mod_q[PEPSI_MAXL];               // B mod q_i

  // round(t d / Q) from Q u B into B
  uint64_t phat_inv[PEPSI_MAXP], phat_inv_shoup[PEPSI_MAXP];   // ((QB)/p)^-1 mod p
  Fix128 theta[PEPSI_MAXL];                   // floor(frac(t B / q_i) * 2^128)
  uint64_t omega_mod_b[PEPSI_MAXL][PEPSI_MAXK];// floor(t B / q_i) mod b_j
  uint64_t tbhat_mod_b[PEPSI_MAXK];           // t (B/b_j) mod b_j
  uint64_t tb_mod_q[PEPSI_MAXL];              // t B mod q_i

  // decryption: round(t x / Q)
  Fix128 t_over_q[PEPSI_MAXL];                // floor(t 2^128 / q_i)
  uint64_t t_mod_q[PEPSI_MAXL];

  // multiword constants of the exact (multi-precision) path
  MWord Qw, Bw;                               // Q, B
  MWord qhat_w[PEPSI_MAXL], bhat_w[PEPSI_MAXK];// Q/q_i, B/b_j

  // modulus switching to q_0 over Q' = q_1 ... q_{L-1} (entry i - 1 for prime q_i)
  MWord sw_hat_w[PEPSI_MAXL], sw_Qw;          // Q'/q_i, Q'
  uint64_t sw_hat_inv[PEPSI_MAXL];            // (Q'/q_i)^-1 mod q_i
  uint64_t sw_hat_mod_q0[PEPSI_MAXL];         // (Q'/q_i) mod q_0
  uint64_t sw_q_mod_q0, sw_qinv_q0;           // Q' mod q_0, Q'^-1 mod q_0
};

// Device-resident tables (all device pointers).
struct Tables {
  const Consts* c;                 // the struct above
  const uint64_t* psi_rev;         // [L+K][N]  psi^brv(k)
  const uint64_t* psi_rev_shoup;   // [L+K][N]
  const uint64_t* ipsi_rev;        // [L+K][N]  psi^-brv(k)
  const uint64_t* ipsi_rev_shoup;  // [L+K][N]
  const uint32_t* psit_rev;        // [N]  psi_t^brv(k)
  const uint32_t* ipsit_rev;       // [N]  psi_t^-brv(k)
};

// Host-side description, built once per parameter set.
struct HostParams {
  int n, logn, L, K;
  int h, ell, mu, item_bits, n_hash, max_evictions;
  int pbh, eff_bits;   // permutation-based hashing; length of the stored values (lambda_bar)
  uint64_t hash_seed;
  uint64_t primes[PEPSI_MAXP];
  uint64_t psi[PEPSI_MAXP];
  uint32_t psi_t;
  Consts consts;
};

// Builds every constant; returns 0 or a negative status with a message.
int build_host_params(int logn, int L, int h, int item_bits, int mu, int n_hash,
                      uint64_t hash_seed, int max_evictions, int pbh, HostParams* out,
                      char* err, int errlen);
