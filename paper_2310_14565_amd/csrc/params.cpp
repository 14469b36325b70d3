// Host construction of the scheme constants (primes, roots, RNS tables).
#include "params.hpp"

#include <stdio.h>
#include <string.h>

namespace {

uint64_t mulm(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)(((u128)a * b) % m); }
uint64_t powm(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  for (; e; e >>= 1) {
    if (e & 1) r = mulm(r, a, m);
    a = mulm(a, a, m);
  }
  return r;
}
uint64_t invm(uint64_t a, uint64_t m) { return powm(a % m, m - 2, m); }

bool is_prime(uint64_t n) {
  if (n < 2) return false;
  static const uint64_t small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (uint64_t p : small)
    if (n % p == 0) return n == p;
  uint64_t d = n - 1;
  int s = 0;
  while ((d & 1) == 0) { d >>= 1; ++s; }
  for (uint64_t a : small) {
    uint64_t x = powm(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s; ++r) {
      x = mulm(x, x, n);
      if (x == n - 1) { comp = false; break; }
    }
    if (comp) return false;
  }
  return true;
}

// psi = c^((p-1)/2n) for the least quadratic non-residue c: psi^n = -1.
uint64_t root_2n(uint64_t p, uint64_t n) {
  uint64_t c = 2;
  while (powm(c, (p - 1) / 2, p) != p - 1) ++c;
  return powm(c, (p - 1) / (2 * n), p);
}

// floor(num * 2^128 / q) for num < q, as two words.
Fix128 frac128(uint64_t num, uint64_t q) {
  u128 x = (u128)num << 64;
  uint64_t a1 = (uint64_t)(x / q);
  uint64_t r1 = (uint64_t)(x % q);
  u128 y = (u128)r1 << 64;
  uint64_t a0 = (uint64_t)(y / q);
  return Fix128{a0, a1};
}

// little multiword helpers on PEPSI_MW words
void mw_set(MWord& a, uint64_t v) { memset(a.w, 0, sizeof(a.w)); a.w[0] = v; }
bool mw_mul_small(MWord& a, uint64_t v) {
  u128 c = 0;
  for (int i = 0; i < PEPSI_MW; ++i) {
    c += (u128)a.w[i] * v;
    a.w[i] = (uint64_t)c;
    c >>= 64;
  }
  return c == 0;
}
uint64_t mw_mod_small(const MWord& a, uint64_t m) {
  u128 r = 0;
  for (int i = PEPSI_MW - 1; i >= 0; --i) r = ((r << 64) | a.w[i]) % m;
  return (uint64_t)r;
}
MWord mw_div_small(const MWord& a, uint64_t m) {
  MWord q;
  u128 r = 0;
  for (int i = PEPSI_MW - 1; i >= 0; --i) {
    r = (r << 64) | a.w[i];
    q.w[i] = (uint64_t)(r / m);
    r %= m;
  }
  return q;
}
int mw_bits(const MWord& a) {
  for (int i = PEPSI_MW - 1; i >= 0; --i)
    if (a.w[i]) return 64 * i + 64 - __builtin_clzll(a.w[i]);
  return 0;
}

Prime make_prime(uint64_t p) {
  Prime P;
  P.p = p;
  P.barrett = (uint64_t)(((u128)1 << 116) / p);
  P.r64 = (uint64_t)(((u128)1 << 64) % p);
  return P;
}

}  // namespace

int build_host_params(int logn, int L, int h, int item_bits, int mu, int n_hash,
                      uint64_t hash_seed, int max_evictions, int pbh, HostParams* out,
                      char* err, int errlen) {
  if (logn < 10 || logn > 14) { snprintf(err, errlen, "log_n must be in [10, 14]"); return -2; }
  if (L < 1 || L > PEPSI_MAXL) { snprintf(err, errlen, "n_q must be in [1, %d]", PEPSI_MAXL); return -2; }
  if (h < 1 || h > 16) { snprintf(err, errlen, "h must be in [1, 16]"); return -2; }
  if (item_bits < 1 || item_bits > 64) { snprintf(err, errlen, "item_bits must be in [1, 64]"); return -2; }
  if (mu < 1) { snprintf(err, errlen, "mu must be positive"); return -2; }
  if (n_hash < 1 || n_hash > 8) { snprintf(err, errlen, "n_hash must be in [1, 8]"); return -2; }
  HostParams& H = *out;
  memset(&H, 0, sizeof(H));
  const int n = 1 << logn;
  const int K = L + 1;
  H.n = n; H.logn = logn; H.L = L; H.K = K;
  H.h = h; H.item_bits = item_bits; H.mu = mu; H.n_hash = n_hash;
  // stored values: the element, or with PBH lambda - log2 N bits plus the hash-function index
  H.pbh = pbh ? 1 : 0;
  H.eff_bits = item_bits;
  if (pbh) {
    int ib = 0;
    while ((1 << ib) < n_hash) ++ib;
    if (item_bits <= logn) { snprintf(err, errlen, "PBH needs item_bits > log_n"); return -2; }
    H.eff_bits = item_bits - logn + ib;
    if (H.eff_bits > 64) { snprintf(err, errlen, "PBH values exceed 64 bits"); return -2; }
  }
  H.hash_seed = hash_seed; H.max_evictions = max_evictions;

  // code length, eq. (1): least l with C(l, h) >= 2^lambda_bar (C(l, h) grows with l, and
  // every C(l, r), r <= h, stays below the target until the answer, so u128 cannot overflow)
  {
    const u128 target = (u128)1 << H.eff_bits;
    int ell = h;
    for (;; ++ell) {
      if (ell > 0xFFFE) { snprintf(err, errlen, "code length exceeds 65534"); return -2; }
      u128 c = 1;
      for (int r = 0; r < h; ++r) c = c * (u128)(ell - r) / (u128)(r + 1);   // C(ell, r+1)
      if (c >= target) break;
    }
    H.ell = ell;
  }

  // primes: the largest below 2^54 with p = 1 mod 2n, descending; Q first, then B
  {
    const uint64_t step = 2 * (uint64_t)n;
    uint64_t q = (((uint64_t)1 << 54) - 1) / step * step + 1;
    if (q >= ((uint64_t)1 << 54)) q -= step;
    int got = 0;
    while (got < L + K) {
      if (is_prime(q)) H.primes[got++] = q;
      q -= step;
    }
    for (int i = 0; i < L + K; ++i) H.psi[i] = root_2n(H.primes[i], n);
    H.psi_t = (uint32_t)root_2n(PEPSI_T, n);
  }

  Consts& C = H.consts;
  C.n = n; C.logn = logn; C.L = L; C.K = K;
  for (int i = 0; i < L + K; ++i) {
    uint64_t p = H.primes[i];
    C.prm[i] = make_prime(p);
    C.n_inv[i] = invm(n, p);
    C.n_inv_shoup[i] = shoup_companion(C.n_inv[i], p);
  }
  C.n_inv_t = (uint32_t)invm(n, PEPSI_T);

  const uint64_t* q = H.primes;
  const uint64_t* b = H.primes + L;
  MWord Qw, Bw;
  mw_set(Qw, 1);
  mw_set(Bw, 1);
  for (int i = 0; i < L; ++i) mw_mul_small(Qw, q[i]);
  for (int j = 0; j < K; ++j) mw_mul_small(Bw, b[j]);
  C.Qw = Qw;
  C.Bw = Bw;
  const int qbits = mw_bits(Qw), bbits = mw_bits(Bw);
  if (bbits <= 17 + logn + qbits + 2) {
    snprintf(err, errlen, "auxiliary base too small");
    return -2;
  }
  MWord delta = mw_div_small(Qw, PEPSI_T);
  for (int i = 0; i < L; ++i) C.delta[i] = mw_mod_small(delta, q[i]);

  // Q -> B
  for (int i = 0; i < L; ++i) {
    MWord qh; mw_set(qh, 1);
    for (int k = 0; k < L; ++k) if (k != i) mw_mul_small(qh, q[k]);
    C.qhat_w[i] = qh;
    C.qhat_mod_q[i] = mw_mod_small(qh, q[i]);
    C.qhat_inv[i] = invm(C.qhat_mod_q[i], q[i]);
    C.qhat_inv_shoup[i] = shoup_companion(C.qhat_inv[i], q[i]);
    C.inv_q_d[i] = 1.0 / (double)q[i];
    for (int j = 0; j < K; ++j) C.qhat_mod_b[i][j] = mw_mod_small(qh, b[j]);
  }
  for (int j = 0; j < K; ++j) C.q_mod_b[j] = mw_mod_small(Qw, b[j]);

  // B -> Q
  for (int j = 0; j < K; ++j) {
    MWord bh; mw_set(bh, 1);
    for (int k = 0; k < K; ++k) if (k != j) mw_mul_small(bh, b[k]);
    C.bhat_w[j] = bh;
    C.bhat_inv[j] = invm(mw_mod_small(bh, b[j]), b[j]);
    C.bhat_inv_shoup[j] = shoup_companion(C.bhat_inv[j], b[j]);
    C.inv_b_d[j] = 1.0 / (double)b[j];
    for (int i = 0; i < L; ++i) C.bhat_mod_q[j][i] = mw_mod_small(bh, q[i]);
  }
  for (int i = 0; i < L; ++i) C.b_mod_q[i] = mw_mod_small(Bw, q[i]);

  // scale and round: over P = Q B
  for (int i = 0; i < L + K; ++i) {
    uint64_t p = H.primes[i];
    uint64_t prod = 1;
    for (int k = 0; k < L + K; ++k) if (k != i) prod = mulm(prod, H.primes[k] % p, p);
    C.phat_inv[i] = invm(prod, p);
    C.phat_inv_shoup[i] = shoup_companion(C.phat_inv[i], p);
  }
  for (int i = 0; i < L; ++i) {
    uint64_t r = mulm(PEPSI_T, mw_mod_small(Bw, q[i]), q[i]);        // t B mod q_i
    C.tb_mod_q[i] = r;
    C.theta[i] = frac128(r, q[i]);
    for (int j = 0; j < K; ++j) {
      // floor(tB/q_i) = (tB - r)/q_i and tB = 0 mod b_j, so it is -r * q_i^-1 mod b_j
      uint64_t rb = r % b[j];
      uint64_t neg = rb == 0 ? 0 : b[j] - rb;
      C.omega_mod_b[i][j] = mulm(neg, invm(q[i] % b[j], b[j]), b[j]);
    }
  }
  for (int j = 0; j < K; ++j) {
    uint64_t prod = 1;
    for (int k = 0; k < K; ++k) if (k != j) prod = mulm(prod, b[k] % b[j], b[j]);
    C.tbhat_mod_b[j] = mulm(PEPSI_T, prod, b[j]);
  }

  // decryption
  for (int i = 0; i < L; ++i) {
    C.t_over_q[i] = frac128(PEPSI_T, q[i]);
    C.t_mod_q[i] = PEPSI_T % q[i];
  }

  // modulus switching to q_0
  mw_set(C.sw_Qw, 1);
  for (int i = 1; i < L; ++i) mw_mul_small(C.sw_Qw, q[i]);
  for (int i = 1; i < L; ++i) {
    MWord h; mw_set(h, 1);
    for (int k = 1; k < L; ++k) if (k != i) mw_mul_small(h, q[k]);
    C.sw_hat_w[i - 1] = h;
    C.sw_hat_inv[i - 1] = invm(mw_mod_small(h, q[i]), q[i]);
    C.sw_hat_mod_q0[i - 1] = mw_mod_small(h, q[0]);
  }
  C.sw_q_mod_q0 = mw_mod_small(C.sw_Qw, q[0]);
  C.sw_qinv_q0 = invm(C.sw_q_mod_q0, q[0]);
  return 0;
}
