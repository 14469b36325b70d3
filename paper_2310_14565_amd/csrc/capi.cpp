// C-ABI of the PEPSI server computation on gfx950 (see include/pepsi.h).
#include "../../include/pepsi.h"

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "kernels.hpp"
#include "params.hpp"
#include "protocol.hpp"

using namespace pepsi;

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(PEPSI_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
  } while (0)

inline hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

// Device buffer that only grows; growing waits for the device first.
// Device buffer owned by value: grows on demand, freed with its owner.
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), cap(o.cap) { o.p = nullptr; o.cap = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      cap = o.cap;
      o.p = nullptr;
      o.cap = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  int ensure(size_t bytes) {
    if (bytes <= cap) return 0;
    if (p) {
      HIPCHK(hipDeviceSynchronize());
      HIPCHK(hipFree(p));
      p = nullptr;
      cap = 0;
    }
    if (hipMalloc(&p, bytes) != hipSuccess) {
      p = nullptr;
      return fail(PEPSI_E_NOMEM, "hipMalloc of %zu bytes failed", bytes);
    }
    cap = bytes;
    return 0;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  template <class T> T* as(size_t word_offset = 0) const {
    return reinterpret_cast<T*>(p) + word_offset;
  }
};
}  // namespace

extern "C" const char* pepsi_last_error(void) { return g_err.c_str(); }

// ------------------------------------------------------------------ params
struct pepsi_params {
  HostParams H;
  int device = 0;
  Tables T{};
  DevBuf consts, tw, twt, fallback;
  DevBuf scratch;                 // single-step operations
  std::vector<TensorJob> one_job;
  DevBuf job_dev;
  size_t words_poly() const { return (size_t)H.n; }
};

namespace {

uint64_t powm(uint64_t a, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  a %= m;
  for (; e; e >>= 1) {
    if (e & 1) r = (uint64_t)(((u128)r * a) % m);
    a = (uint64_t)(((u128)a * a) % m);
  }
  return r;
}
uint32_t brv(uint32_t k, int logn) {
  uint32_t r = 0;
  for (int i = 0; i < logn; ++i) r |= ((k >> i) & 1u) << (logn - 1 - i);
  return r;
}

int upload_tables(pepsi_params* P) {
  const HostParams& H = P->H;
  const int n = H.n, np = H.L + H.K;
  std::vector<uint64_t> tw((size_t)4 * np * n);
  uint64_t* psi_rev = tw.data();
  uint64_t* psi_rev_q = psi_rev + (size_t)np * n;
  uint64_t* ipsi_rev = psi_rev_q + (size_t)np * n;
  uint64_t* ipsi_rev_q = ipsi_rev + (size_t)np * n;
  for (int i = 0; i < np; ++i) {
    const uint64_t p = H.primes[i];
    const uint64_t psi = H.psi[i], ipsi = powm(psi, p - 2, p);
    for (int k = 0; k < n; ++k) {
      const uint64_t e = brv(k, H.logn);
      const uint64_t w = powm(psi, e, p), iw = powm(ipsi, e, p);
      psi_rev[(size_t)i * n + k] = w;
      psi_rev_q[(size_t)i * n + k] = shoup_companion(w, p);
      ipsi_rev[(size_t)i * n + k] = iw;
      ipsi_rev_q[(size_t)i * n + k] = shoup_companion(iw, p);
    }
  }
  std::vector<uint32_t> twt((size_t)2 * n);
  const uint64_t ipt = powm(H.psi_t, PEPSI_T - 2, PEPSI_T);
  for (int k = 0; k < n; ++k) {
    const uint64_t e = brv(k, H.logn);
    twt[k] = (uint32_t)powm(H.psi_t, e, PEPSI_T);
    twt[n + k] = (uint32_t)powm(ipt, e, PEPSI_T);
  }
  int rc;
  if ((rc = P->consts.ensure(sizeof(Consts)))) return rc;
  if ((rc = P->tw.ensure(tw.size() * 8))) return rc;
  if ((rc = P->twt.ensure(twt.size() * 4))) return rc;
  if ((rc = P->fallback.ensure(64))) return rc;
  HIPCHK(hipMemcpy(P->consts.p, &H.consts, sizeof(Consts), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(P->tw.p, tw.data(), tw.size() * 8, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(P->twt.p, twt.data(), twt.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(hipMemset(P->fallback.p, 0, 64));
  P->T.c = P->consts.as<Consts>();
  P->T.psi_rev = P->tw.as<uint64_t>();
  P->T.psi_rev_shoup = P->tw.as<uint64_t>((size_t)np * n);
  P->T.ipsi_rev = P->tw.as<uint64_t>((size_t)2 * np * n);
  P->T.ipsi_rev_shoup = P->tw.as<uint64_t>((size_t)3 * np * n);
  P->T.psit_rev = P->twt.as<uint32_t>();
  P->T.ipsit_rev = P->twt.as<uint32_t>(n);
  return 0;
}

}  // namespace

extern "C" int pepsi_params_create(const pepsi_params_desc* d, pepsi_params** out) {
  if (!d || !out) return fail(PEPSI_E_ARG, "null argument");
  *out = nullptr;
  if (d->flags & ~PEPSI_PARAMS_PBH) return fail(PEPSI_E_ARG, "unknown flags");
  pepsi_params* P = new pepsi_params();
  char err[256] = {0};
  int rc = build_host_params((int)d->log_n, (int)d->n_q, (int)d->h, (int)d->item_bits, (int)d->mu,
                             (int)d->n_hash, d->hash_seed, (int)d->max_evictions,
                             (d->flags & PEPSI_PARAMS_PBH) ? 1 : 0, &P->H, err,
                             sizeof(err));
  if (rc) {
    delete P;
    return fail(rc, "%s", err);
  }
  if (hipGetDevice(&P->device) != hipSuccess) {
    delete P;
    return fail(PEPSI_E_DEVICE, "no HIP device");
  }
  if ((rc = upload_tables(P))) {
    std::string msg = g_err;
    pepsi_params_destroy(P);
    return fail(rc, "%s", msg.c_str());
  }
  *out = P;
  return PEPSI_OK;
}

extern "C" int pepsi_params_get_info(const pepsi_params* P, pepsi_params_info* o) {
  if (!P || !o) return fail(PEPSI_E_ARG, "null argument");
  const HostParams& H = P->H;
  memset(o, 0, sizeof(*o));
  o->n = H.n; o->n_q = H.L; o->n_aux = H.K; o->h = H.h; o->ell = H.ell; o->mu = H.mu;
  o->item_bits = H.item_bits; o->n_hash = H.n_hash; o->t = PEPSI_T;
  for (int i = 0; i < H.L + H.K; ++i) { o->primes[i] = H.primes[i]; o->psi[i] = H.psi[i]; }
  o->psi_t = H.psi_t;
  int bits = 0;
  for (int w = PEPSI_MW - 1; w >= 0; --w)
    if (H.consts.Qw.w[w]) { bits = 64 * w + 64 - __builtin_clzll(H.consts.Qw.w[w]); break; }
  o->q_bits = bits;
  const uint64_t n = H.n, L = H.L;
  o->ct_bytes = 2 * L * n * 8;
  o->query_bytes = (uint64_t)H.ell * o->ct_bytes;
  o->rlk_bytes = L * o->ct_bytes;
  o->cache_bytes = (uint64_t)H.mu * H.ell * L * n * 8;
  o->effective_bits = (uint32_t)H.eff_bits;
  o->flags = H.pbh ? PEPSI_PARAMS_PBH : 0u;
  return PEPSI_OK;
}

extern "C" void pepsi_params_destroy(pepsi_params* P) {
  if (!P) return;
  (void)hipDeviceSynchronize();
  P->consts.release(); P->tw.release(); P->twt.release(); P->fallback.release();
  P->scratch.release(); P->job_dev.release();
  delete P;
}

extern "C" int pepsi_exact_path_count(const pepsi_params* P, uint64_t* out) {
  if (!P || !out) return fail(PEPSI_E_ARG, "null argument");
  uint32_t v = 0;
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipMemcpy(&v, P->fallback.p, 4, hipMemcpyDeviceToHost));
  *out = v;
  return PEPSI_OK;
}

// ------------------------------------------------------------------ client preparation
namespace {
int client_table_impl(const pepsi_params* P, const uint64_t* items, uint64_t m, uint64_t* table, uint8_t* valid) {
  const HostParams& H = P->H;
  std::unordered_set<uint64_t> seen;
  seen.reserve(m * 2);
  for (uint64_t i = 0; i < m; ++i) {
    if (H.item_bits < 64 && (items[i] >> H.item_bits)) return fail(PEPSI_E_RANGE, "item %llu out of range", (unsigned long long)i);
    if (!seen.insert(items[i]).second) return fail(PEPSI_E_RANGE, "duplicate client item");
  }
  if (m > (uint64_t)H.n) return fail(PEPSI_E_CUCKOO, "more items than bins");
  if (cuckoo_insert(items, m, H.n, H.hash_seed, H.n_hash, H.max_evictions, table, valid,
                    H.pbh ? H.item_bits : 0))
    return fail(PEPSI_E_CUCKOO, "cuckoo insertion exceeded %d evictions", H.max_evictions);
  return PEPSI_OK;
}

template <class V>
int codeword_planes_impl(const pepsi_params* P, const V* table, const uint8_t* valid, uint32_t* planes) {
  const HostParams& H = P->H;
  CwEncoder enc(H.ell, H.h);
  memset(planes, 0, sizeof(uint32_t) * (size_t)H.ell * H.n);
  std::vector<uint16_t> pos(H.h);
  for (int k = 0; k < H.n; ++k) {
    if (!valid[k]) continue;
    const uint64_t v = table[k];
    if (H.eff_bits < 64 && (v >> H.eff_bits)) return fail(PEPSI_E_RANGE, "value out of range");
    enc.encode(v, pos.data());
    for (int r = 0; r < H.h; ++r) planes[(size_t)pos[r] * H.n + k] = 1;
  }
  return PEPSI_OK;
}
}  // namespace

extern "C" int pepsi_client_table(const pepsi_params* P, const uint32_t* items, uint64_t m,
                                  uint32_t* table, uint8_t* valid) {
  if (!P || (!items && m) || !table || !valid) return fail(PEPSI_E_ARG, "null argument");
  if (P->H.eff_bits > 32) return fail(PEPSI_E_ARG, "stored values exceed 32 bits: use pepsi_client_table64");
  std::vector<uint64_t> wide(items, items + m), t64(P->H.n);
  const int rc = client_table_impl(P, wide.data(), m, t64.data(), valid);
  if (rc) return rc;
  for (int k = 0; k < P->H.n; ++k) table[k] = (uint32_t)t64[k];
  return PEPSI_OK;
}

extern "C" int pepsi_client_table64(const pepsi_params* P, const uint64_t* items, uint64_t m, uint64_t* table,
                                    uint8_t* valid) {
  if (!P || (!items && m) || !table || !valid) return fail(PEPSI_E_ARG, "null argument");
  return client_table_impl(P, items, m, table, valid);
}

extern "C" int pepsi_codeword_planes(const pepsi_params* P, const uint32_t* table, const uint8_t* valid,
                                     uint32_t* planes) {
  if (!P || !table || !valid || !planes) return fail(PEPSI_E_ARG, "null argument");
  return codeword_planes_impl(P, table, valid, planes);
}

extern "C" int pepsi_codeword_planes64(const pepsi_params* P, const uint64_t* table, const uint8_t* valid,
                                       uint32_t* planes) {
  if (!P || !table || !valid || !planes) return fail(PEPSI_E_ARG, "null argument");
  return codeword_planes_impl(P, table, valid, planes);
}

// ------------------------------------------------------------------ large elements
extern "C" int pepsi_large_element_bits(uint32_t n_bins, uint32_t mu_client, uint32_t mu_server, uint32_t alpha,
                                        uint32_t* bits) {
  if (!bits) return fail(PEPSI_E_ARG, "null argument");
  if (!n_bins || !mu_client || !mu_server) return fail(PEPSI_E_ARG, "bins and bin loads must be positive");
  const u128 x = (u128)n_bins * mu_client * mu_server;
  uint32_t c = 0;                                  // ceil(log2 x)
  while (((u128)1 << c) < x) ++c;
  *bits = alpha + c;
  return PEPSI_OK;
}

extern "C" int pepsi_hash_elements(uint32_t bits, const uint8_t* data, const uint64_t* offsets, uint64_t count,
                                   uint64_t* out) {
  if ((!data && count) || (!offsets && count) || (!out && count)) return fail(PEPSI_E_ARG, "null argument");
  if (bits < 1 || bits > 64) return fail(PEPSI_E_ARG, "bits must be in [1, 64]");
  for (uint64_t e = 0; e < count; ++e) {
    if (offsets[e + 1] < offsets[e]) return fail(PEPSI_E_ARG, "offsets must not decrease");
    out[e] = hash_element(data + offsets[e], offsets[e + 1] - offsets[e], (int)bits);
  }
  return PEPSI_OK;
}

// ------------------------------------------------------------------ keys and encryption
extern "C" int pepsi_encrypt(const pepsi_params* Pc, const int8_t* sk, const uint32_t* slots,
                             const uint64_t* a, const int32_t* e, uint32_t count, uint64_t* ct,
                             void* stream) {
  pepsi_params* P = const_cast<pepsi_params*>(Pc);
  if (!P || !sk || !slots || !a || !e || !ct) return fail(PEPSI_E_ARG, "null argument");
  if (!count) return PEPSI_OK;
  const HostParams& H = P->H;
  const size_t n = H.n, L = H.L;
  // scratch: m (u32 count*n) | ahat (count*L*n) | shat (L*n)
  const size_t w_m = (count * n + 1) / 2, w_ah = count * L * n, w_sh = L * n;
  int rc = P->scratch.ensure((w_m + w_ah + w_sh) * 8);
  if (rc) return rc;
  uint32_t* m = P->scratch.as<uint32_t>();
  uint64_t* ah = P->scratch.as<uint64_t>(w_m);
  uint64_t* sh = ah + w_ah;
  hipStream_t s = S(stream);
  encode_slots(P->T, H.logn, slots, m, count, s);
  ntt_forward(P->T, H.logn, a, LOAD_U64, ah, STORE_U64, (int)(count * L), (int)L, 0, s);
  ntt_forward(P->T, H.logn, sk, LOAD_I8, sh, STORE_U64, (int)L, (int)L, 0, s);
  pointwise_mul(P->T, H.consts, ah, sh, ah, (int)count, (int)L, true, s);
  ntt_inverse(P->T, H.logn, ah, ah, (int)(count * L), (int)L, 0, s);
  encrypt_finish(P->T, H.consts, m, ah, e, a, ct, (int)count, s);
  HIPCHK(hipGetLastError());
  return PEPSI_OK;
}

extern "C" int pepsi_keygen_relin(const pepsi_params* Pc, const int8_t* sk, const uint64_t* a,
                                  const int32_t* e, uint64_t* rlk, void* stream) {
  pepsi_params* P = const_cast<pepsi_params*>(Pc);
  if (!P || !sk || !a || !e || !rlk) return fail(PEPSI_E_ARG, "null argument");
  const HostParams& H = P->H;
  const size_t n = H.n, L = H.L;
  // scratch: shat (L n) | s2 (L n) | as (L L n)
  int rc = P->scratch.ensure((2 * L * n + L * L * n) * 8);
  if (rc) return rc;
  uint64_t* sh = P->scratch.as<uint64_t>();
  uint64_t* s2 = sh + L * n;
  uint64_t* as = s2 + L * n;
  hipStream_t s = S(stream);
  ntt_forward(P->T, H.logn, sk, LOAD_I8, sh, STORE_U64, (int)L, (int)L, 0, s);
  pointwise_mul(P->T, H.consts, sh, sh, s2, 1, (int)L, false, s);
  ntt_inverse(P->T, H.logn, s2, s2, (int)L, (int)L, 0, s);
  ntt_forward(P->T, H.logn, a, LOAD_U64, as, STORE_U64, (int)(L * L), (int)L, 0, s);
  pointwise_mul(P->T, H.consts, as, sh, as, (int)L, (int)L, true, s);
  ntt_inverse(P->T, H.logn, as, as, (int)(L * L), (int)L, 0, s);
  keygen_finish(P->T, H.consts, s2, as, e, a, rlk, s);
  HIPCHK(hipGetLastError());
  return PEPSI_OK;
}

namespace {
// x = c0 + c1 s (coefficient form) for count ciphertexts into scratch; returns pointer
int phase_coeff(pepsi_params* P, const int8_t* sk, const uint64_t* ct, uint32_t count, uint64_t** x_out,
                size_t extra_words, hipStream_t s) {
  const HostParams& H = P->H;
  const size_t n = H.n, L = H.L;
  const size_t w_ch = count * 2 * L * n, w_sh = L * n, w_x = count * L * n;
  int rc = P->scratch.ensure((w_ch + w_sh + w_x + extra_words) * 8);
  if (rc) return rc;
  uint64_t* ch = P->scratch.as<uint64_t>();
  uint64_t* sh = ch + w_ch;
  uint64_t* x = sh + w_sh;
  ntt_forward(P->T, H.logn, ct, LOAD_U64, ch, STORE_U64, (int)(count * 2 * L), (int)L, 0, s);
  ntt_forward(P->T, H.logn, sk, LOAD_I8, sh, STORE_U64, (int)L, (int)L, 0, s);
  phase_ntt(P->T, H.consts, ch, sh, x, (int)count, s);
  ntt_inverse(P->T, H.logn, x, x, (int)(count * L), (int)L, 0, s);
  *x_out = x;
  return 0;
}
}  // namespace

extern "C" int pepsi_decrypt(const pepsi_params* Pc, const int8_t* sk, const uint64_t* ct,
                             uint32_t count, uint32_t* slots, void* stream) {
  pepsi_params* P = const_cast<pepsi_params*>(Pc);
  if (!P || !sk || !ct || !slots) return fail(PEPSI_E_ARG, "null argument");
  if (!count) return PEPSI_OK;
  const HostParams& H = P->H;
  hipStream_t s = S(stream);
  uint64_t* x;
  const size_t w_m = (count * (size_t)H.n + 1) / 2;
  int rc = phase_coeff(P, sk, ct, count, &x, w_m, s);
  if (rc) return rc;
  uint32_t* m = reinterpret_cast<uint32_t*>(x + (size_t)count * H.L * H.n);
  decrypt_round(P->T, H.consts, x, m, (int)count, P->fallback.as<uint32_t>(), s);
  decode_slots(P->T, H.logn, m, slots, (int)count, s);
  HIPCHK(hipGetLastError());
  return PEPSI_OK;
}

extern "C" int pepsi_noise_budget(const pepsi_params* Pc, const int8_t* sk, const uint64_t* ct,
                                  int32_t* budget, void* stream) {
  pepsi_params* P = const_cast<pepsi_params*>(Pc);
  if (!P || !sk || !ct || !budget) return fail(PEPSI_E_ARG, "null argument");
  hipStream_t s = S(stream);
  uint64_t* x;
  int rc = phase_coeff(P, sk, ct, 1, &x, 1, s);
  if (rc) return rc;
  uint32_t* bits = reinterpret_cast<uint32_t*>(x + (size_t)P->H.L * P->H.n);
  HIPCHK(hipMemsetAsync(bits, 0, 4, s));
  noise_bits(P->T, P->H.consts, x, 1, bits, s);
  uint32_t hb = 0;
  HIPCHK(hipMemcpyAsync(&hb, bits, 4, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  pepsi_params_info info;
  pepsi_params_get_info(P, &info);
  *budget = (int32_t)info.q_bits - (int32_t)hb - 1;
  return PEPSI_OK;
}

// ------------------------------------------------------------------ evaluation engine
namespace {

struct EventTimer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  struct Pend { hipEvent_t a, b; int kind; uint64_t bytes; };
  std::vector<Pend> pending;
  pepsi_timing tot{};
  hipEvent_t get() {
    if (pool.empty()) {
      hipEvent_t e;
      (void)hipEventCreate(&e);
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  int fold() {
    for (auto& p : pending) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) return -1;
      if (p.kind == 0) { tot.select_sum_launches++; tot.select_sum_ms += ms; tot.select_sum_bytes += p.bytes; }
      else if (p.kind == 2) { tot.ntt_fwd_launches++; tot.ntt_fwd_ms += ms; tot.ntt_fwd_rows += p.bytes; }
      else if (p.kind == 3) { tot.ntt_inv_launches++; tot.ntt_inv_ms += ms; tot.ntt_inv_rows += p.bytes; }
      else if (p.kind == 4) { tot.rescale_launches++; tot.rescale_ms += ms; tot.rescale_products += p.bytes; }
      else if (p.kind == 5) { tot.ext_launches++; tot.ext_ms += ms; tot.ext_products += p.bytes; }
      else { tot.evals++; tot.eval_ms += ms; }
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
    return 0;
  }
  ~EventTimer() {
    for (auto& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};


struct Operand { const uint64_t* q; const uint64_t* b; const uint64_t* alpha; };

// Workspace of the server computation for up to Qmax queries at once.  A tile is TBq server
// batches of every query; the (batch b, query q) "pair" p = b * nq + q carries one
// select-and-sum ciphertext through the product tree.  Pairs are batch-major, so a partial
// tile of nb batches uses the first nb * nq pairs (and the first jobs of every tree level).
struct Engine {
  pepsi_params* P = nullptr;
  int TBq = 0, Qmax = 0, levels = 0;
  std::vector<int> jobs_at;            // tensor jobs per pair at each tree level
  DevBuf chat, rlkhat, acc, accD;      // per query: request and key in NTT form, running sums
  DevBuf sq, scoef, sb, sbh, alpha, pconst, e; // per pair: S over Q (NTT, coefficients), over B (both), ...
  DevBuf d, c01, c01h, c2, D, rcoef;   // per tensor job
  std::vector<DevBuf> rq, rb;          // per tree level outputs
  DevBuf jobs;                         // device TensorJob arrays, all levels
  DevBuf gen_poly, gen_p;              // on-the-fly plaintext generation
  DevBuf cplanes;                      // per query: request digit planes (matrix-core select-and-sum)
  DevBuf sall;                         // select-and-sum outputs of a run of tiles (run mode)
  uint32_t run_cap = 0;                // batches per run (a multiple of TBq and of 16), 0: off
  bool planes_on = false;
  int GB = 0;
  EventTimer* timer = nullptr;
  const uint64_t* vhat = nullptr;      // server-value plaintexts [max_load][L][N] (NTT form) or null

  ~Engine() {
    for (DevBuf* b : {&chat, &rlkhat, &acc, &accD, &sq, &scoef, &sb, &sbh, &alpha, &pconst, &e, &d, &c01, &c01h, &c2, &D,
                      &rcoef, &jobs, &gen_poly, &gen_p, &cplanes, &sall})
      b->release();
    for (auto& b : rq) b.release();
    for (auto& b : rb) b.release();
  }
  // device bytes the workspace holds now (a new setup reuses them)
  size_t held_bytes() const {
    size_t t = 0;
    for (const DevBuf* b : {&chat, &rlkhat, &acc, &accD, &sq, &scoef, &sb, &sbh, &alpha, &pconst, &e, &d, &c01, &c01h,
                            &c2, &D, &rcoef, &jobs, &gen_poly, &gen_p, &cplanes, &sall})
      t += b->cap;
    for (const auto& b : rq) t += b.cap;
    for (const auto& b : rb) t += b.cap;
    return t;
  }

  // Transforms of the engine, event-timed (rows per launch) while the server's timer is on.
  void tfwd(const void* in, void* out, int rows, int nprimes, int first, hipStream_t s, NttLoad ld = LOAD_U64) {
    hipEvent_t a = nullptr, b = nullptr;
    if (timer && timer->on && rows > 0) { a = timer->get(); b = timer->get(); (void)hipEventRecord(a, s); }
    ntt_forward(P->T, P->H.logn, in, ld, out, STORE_U64, rows, nprimes, first, s);
    if (a) { (void)hipEventRecord(b, s); timer->pending.push_back({a, b, 2, (uint64_t)rows}); }
  }
  // inverse transforms of products formed while loading (INV_SQUARES of the pairs' X, or
  // INV_TENSOR of the jobs) into d [units][3][L + K][N]
  void tinv_products(InvProducts mode, const uint64_t* xq, const uint64_t* xb, const TensorJob* jobs, uint64_t* out,
                     int units, hipStream_t s) {
    // not among the timed transforms: their loads form the products, so their rows cost more
    ntt_inverse_products(P->T, P->H.logn, mode, xq, xb, jobs, out, units, P->H.L + P->H.K, s);
  }
  void tinv(const uint64_t* in, uint64_t* out, int rows, int nprimes, int first, hipStream_t s) {
    hipEvent_t a = nullptr, b = nullptr;
    if (timer && timer->on && rows > 0) { a = timer->get(); b = timer->get(); (void)hipEventRecord(a, s); }
    ntt_inverse(P->T, P->H.logn, in, out, rows, nprimes, first, s);
    if (a) { (void)hipEventRecord(b, s); timer->pending.push_back({a, b, 3, (uint64_t)rows}); }
  }
  // A rescale (kind 4) or Q -> B extension (kind 5) launch, event-timed with its 54-bit modular
  // products (as counted in pepsi_timing) while the server's timer is on.
  template <class F>
  void timed_rns(int kind, uint64_t products, hipStream_t s, F&& launch) {
    hipEvent_t a = nullptr, b = nullptr;
    if (timer && timer->on && products > 0) { a = timer->get(); b = timer->get(); (void)hipEventRecord(a, s); }
    launch();
    if (a) { (void)hipEventRecord(b, s); timer->pending.push_back({a, b, kind, products}); }
  }
  // products per coefficient of a rescale (plus L + K with the first level's linear terms) and
  // of an extension
  uint64_t rescale_products() const {
    const uint64_t L = P->H.L, K = P->H.K;
    return (L + K) + K * (L + 1) + K + L * (K + 1);
  }
  uint64_t ext_products() const { return P->H.L + P->H.K * (P->H.L + 1); }

  size_t cstride() const { return (size_t)P->H.ell * 2 * P->H.L * P->H.n; }
  size_t rstride() const { return (size_t)P->H.L * 2 * P->H.L * P->H.n; }
  size_t ctw() const { return (size_t)2 * P->H.L * P->H.n; }
  size_t dtw() const { return (size_t)P->H.L * P->H.L * P->H.n; }

  int setup(pepsi_params* params, int tbq, int qmax, bool need_gen, const uint64_t* values_hat = nullptr) {
    vhat = values_hat;
    planes_on = false;
    run_cap = 0;
    P = params;
    const HostParams& H = P->H;
    const size_t n = H.n, L = H.L, K = H.K, Pn = L + K;
    TBq = tbq;
    Qmax = qmax;
    const size_t PC = (size_t)TBq * Qmax;          // pair capacity
    int rc;
    if ((rc = chat.ensure(Qmax * cstride() * 8))) return rc;
    if ((rc = rlkhat.ensure(Qmax * rstride() * 8))) return rc;
    if ((rc = acc.ensure(Qmax * ctw() * 8))) return rc;
    if ((rc = sq.ensure(PC * 2 * L * n * 8))) return rc;
    // e: the mask's encoding in finish, and with server values each pair's equality ciphertext
    if ((rc = e.ensure(vhat ? PC * 2 * L * n * 8 : n * 8))) return rc;
    jobs_at.clear();
    for (int cnt = H.h; cnt > 1; cnt = cnt / 2 + cnt % 2) jobs_at.push_back(cnt / 2);
    levels = (int)jobs_at.size();
    if (levels > 0) {
      if ((rc = accD.ensure(Qmax * dtw() * 8))) return rc;
      const size_t J = PC * jobs_at[0];
      if ((rc = scoef.ensure(PC * 2 * L * n * 8))) return rc;
      if ((rc = sb.ensure(PC * 2 * K * n * 8))) return rc;
      if ((rc = sbh.ensure(PC * 2 * K * n * 8))) return rc;
      if ((rc = alpha.ensure(PC * H.h * Pn * 8))) return rc;
      if ((rc = pconst.ensure(PC * std::max(1, H.h / 2) * Pn * 2 * 8))) return rc;
      if ((rc = d.ensure(J * 3 * Pn * n * 8))) return rc;
      if ((rc = c01.ensure(J * 2 * L * n * 8))) return rc;
      if ((rc = c01h.ensure(J * 2 * L * n * 8))) return rc;
      if ((rc = c2.ensure(J * L * n * 8))) return rc;
      if ((rc = D.ensure(J * L * L * n * 8))) return rc;
      if ((rc = rcoef.ensure(J * 2 * L * n * 8))) return rc;
      rq.resize(levels);
      rb.resize(levels);
      for (int lv = 0; lv + 1 < levels; ++lv) {
        const size_t Jl = PC * jobs_at[lv];
        if ((rc = rq[lv].ensure(Jl * 2 * L * n * 8))) return rc;
        if ((rc = rb[lv].ensure(Jl * 2 * K * n * 8))) return rc;
      }
    }
    if (need_gen) {
      GB = std::min(TBq, 16);
      if ((rc = gen_poly.ensure((size_t)GB * H.ell * n * 4))) return rc;
      if ((rc = gen_p.ensure((size_t)GB * H.ell * L * n * 8))) return rc;
    }
    return build_all_jobs();
  }

  // Tensor jobs of every level for a full tile of na active queries (job = pair * pairs + u),
  // for every na in [1, Qmax]; job_off[na][lv] locates them in one device array.
  std::vector<std::vector<size_t>> job_off_na;
  int build_all_jobs() {
    if (levels == 0) return 0;
    const HostParams& H = P->H;
    const size_t n = H.n, L = H.L, K = H.K, Pn = L + K;
    std::vector<TensorJob> all;
    job_off_na.assign(Qmax + 1, std::vector<size_t>(levels, 0));
    for (int na = 1; na <= Qmax; ++na) {
      const int npairs = TBq * na;
      std::vector<std::vector<Operand>> ops(npairs);
      for (int p = 0; p < npairs; ++p)
        for (int r = 0; r < H.h; ++r)
          ops[p].push_back(Operand{sq.as<uint64_t>((size_t)p * 2 * L * n), sbh.as<uint64_t>((size_t)p * 2 * K * n),
                                   alpha.as<uint64_t>(((size_t)p * H.h + r) * Pn)});
      for (int lv = 0; lv < levels; ++lv) {
        const int pairs = jobs_at[lv];
        job_off_na[na][lv] = all.size();
        for (int p = 0; p < npairs; ++p)
          for (int u = 0; u < pairs; ++u) {
            const Operand& x = ops[p][2 * u];
            const Operand& y = ops[p][2 * u + 1];
            const size_t j = (size_t)p * pairs + u;
            all.push_back(TensorJob{x.q, x.b, y.q, y.b, x.alpha, y.alpha, d.as<uint64_t>(j * 3 * Pn * n)});
          }
        if (lv + 1 < levels) {
          for (int p = 0; p < npairs; ++p) {
            std::vector<Operand> next;
            for (int u = 0; u < pairs; ++u) {
              const size_t j = (size_t)p * pairs + u;
              next.push_back(Operand{rq[lv].as<uint64_t>(j * 2 * L * n), rb[lv].as<uint64_t>(j * 2 * K * n), nullptr});
            }
            if (ops[p].size() % 2) next.push_back(ops[p].back());
            ops[p] = next;
          }
        }
      }
    }
    int rc = jobs.ensure(all.size() * sizeof(TensorJob));
    if (rc) return rc;
    HIPCHK(hipMemcpy(jobs.p, all.data(), all.size() * sizeof(TensorJob), hipMemcpyHostToDevice));
    return 0;
  }

  // Relinearisation of the products in c01 / c2 (coefficient form) into out [jobs][2][L][N], NTT
  // form: units share one component 2 (jobs_per_unit jobs each); unit / units_per_pair is the
  // pair.  With ext_out also the Q -> B extension of the results, NTT form.
  void relin_stage(int units, int jobs_per_unit, int units_per_pair, int nq, const int* qslot, uint64_t* out,
                   uint64_t* ext_out, hipStream_t s, int key_slot) {
    const HostParams& H = P->H;
    const int L = H.L, K = H.K;
    const int njobs = units * jobs_per_unit;
    // the digits of component 2 are formed while their transform loads c2
    tfwd(c2.p, D.p, units * L * L, L, 0, s, LOAD_DIGITS);
    const uint64_t* key = rlkhat.as<uint64_t>((size_t)key_slot * rstride());
    if (ext_out) {
      // The next level needs the results in coefficient form too (for their extension to B).
      // The jobs of a unit share its key sum K = sum_i D_i rlk_i, so K alone is transformed back
      // (2 L rows per unit) and added to each job's products in coefficient form; the sums are
      // then transformed forward over Q and over B.  (Forming c01 + K in NTT form would need the
      // 2 L rows of c01 forward and of the sum back, per job.)
      uint64_t* kh = c01h.as<uint64_t>();
      relin_inner(P->T, H.consts, nullptr, D.as<uint64_t>(), key, (long)rstride(), qslot, 1, units_per_pair, nq, kh,
                  units, s);
      tinv(kh, kh, units * 2 * L, L, 0, s);
      timed_rns(5, (uint64_t)njobs * 2 * H.n * ext_products(), s, [&] {
        add_ext_q_to_b(P->T, H.consts, c01.as<uint64_t>(), kh, jobs_per_unit, rcoef.as<uint64_t>(), ext_out,
                       njobs * 2, P->fallback.as<uint32_t>(), s);
      });
      tfwd(rcoef.p, out, njobs * 2 * L, L, 0, s);
      tfwd(ext_out, ext_out, njobs * 2 * K, K, L, s);
    } else {
      tfwd(c01.p, c01h.p, njobs * 2 * L, L, 0, s);
      relin_inner(P->T, H.consts, c01h.as<uint64_t>(), D.as<uint64_t>(), key, (long)rstride(), qslot, jobs_per_unit,
                  units_per_pair, nq, out, units, s);
    }
  }

  // First tree level of npairs pairs: the h / 2 products (f_2u, f_2u+1) of each pair share the
  // products of S (formed while their inverse transform loads S), one inverse transform of them
  // and one component 2 (so one relinearisation sum).  Leaves the rescaled products in c01 / c2.
  void first_level(const uint64_t* Sq, int npairs, hipStream_t s) {
    const HostParams& H = P->H;
    uint64_t* dd = d.as<uint64_t>();
    tinv_products(INV_SQUARES, Sq, sbh.as<uint64_t>(), nullptr, dd, npairs, s);
    const uint64_t J0 = H.h / 2;
    const uint64_t prod =
        H.h < 2 ? 0 : (uint64_t)npairs * H.n * ((2 * J0 + 1) * rescale_products() + 2 * J0 * (H.L + H.K));
    timed_rns(4, prod, s, [&] {
      scale_round_first(P->T, H.consts, dd, scoef.as<uint64_t>(), sb.as<uint64_t>(), alpha.as<uint64_t>(),
                        pconst.as<uint64_t>(), H.h, npairs, c01.as<uint64_t>(), c2.as<uint64_t>(),
                        P->fallback.as<uint32_t>(), s);
    });
  }

  // A later tree level: njobs independent products (TensorJob operands, tensored while their
  // inverse transform loads them) into c01 / c2.
  void later_level(const TensorJob* dev_jobs, int njobs, hipStream_t s) {
    const HostParams& H = P->H;
    uint64_t* dd = d.as<uint64_t>();
    tinv_products(INV_TENSOR, nullptr, nullptr, dev_jobs, dd, njobs, s);
    timed_rns(4, (uint64_t)njobs * 3 * H.n * rescale_products(), s, [&] {
      scale_round(P->T, H.consts, dd, c01.as<uint64_t>(), c2.as<uint64_t>(), njobs, P->fallback.as<uint32_t>(), s);
    });
  }

  size_t cpstride() const { return request_plane_bytes(P->H.consts, P->H.ell); }
  // Request digit planes for every query slot, so that tiles whose plaintext planes are resident
  // take the matrix-core select-and-sum.  When they would not fit beside a 2 GiB reserve they
  // stay off, which is an error if the server holds its plaintexts only as planes (required).
  int enable_planes(bool required) {
    planes_on = false;
    if (!planes_supported(P->H.ell)) return 0;
    const size_t need = (size_t)Qmax * cpstride();
    if (need > cplanes.cap) {
      size_t free_b = 0, total_b = 0;
      if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail(PEPSI_E_DEVICE, "hipMemGetInfo failed");
      if (free_b < need + ((size_t)2 << 30))
        return required ? fail(PEPSI_E_NOMEM, "no room for request digit planes (%zu bytes)", need) : 0;
      int rc = cplanes.ensure(need);
      if (rc) return rc;
    }
    planes_on = true;
    return 0;
  }

  // A query enters slot `slot`: request and key to NTT form (and digit planes), running sum to zero.
  void admit(int slot, const uint64_t* cts, const uint64_t* rlk, hipStream_t s) {
    const HostParams& H = P->H;
    const int L = H.L;
    tfwd(cts, chat.as<uint64_t>(slot * cstride()), H.ell * 2 * L, L,
                0, s);
    if (planes_on)
      request_planes(P->T, H.consts, chat.as<uint64_t>(slot * cstride()), H.ell,
                     cplanes.as<int8_t>((size_t)slot * cpstride()), s);
    tfwd(rlk, rlkhat.as<uint64_t>(slot * rstride()), L * 2 * L, L, 0, s);
    zero_words(acc.as<uint64_t>(slot * ctw()), ctw(), s);
    if (levels > 0) zero_words(accD.as<uint64_t>(slot * dtw()), dtw(), s);
  }

  // A run of batches in a plaintext store: batches bfirst .. of a store of groups of gs batches.
  // planes: the digit planes of the tile's 16-batch group, when resident.
  struct PtView { const uint64_t* p = nullptr; int gs = 0, bfirst = 0; const int8_t* planes = nullptr; };
  // Group size of the resident cache of `cached` batches (space is allocated for whole groups).
  static int cache_group(uint32_t cached) { return cached < (uint32_t)PT_GROUP ? (int)cached : PT_GROUP; }

  void timed_select_sum(const PtView& pv, int nb, int nq, const int* qslot, int single_slot, uint64_t* Sx,
                        hipStream_t s) {
    const HostParams& H = P->H;
    const size_t n = H.n, L = H.L;
    hipEvent_t a = nullptr, b = nullptr;
    if (timer && timer->on) { a = timer->get(); b = timer->get(); (void)hipEventRecord(a, s); }
    if (nq == 1 && pv.p) {
      select_sum(P->T, H.consts, chat.as<uint64_t>((size_t)single_slot * cstride()), pv.p, pv.gs, pv.bfirst,
                 H.ell, nb, Sx, (long)(2 * L * n), s);
    } else if (pv.planes && planes_on) {
      // at most 4 groups per launch; a single query reads its planes from its own slot
      const size_t gbytes = plaintext_plane_group_bytes(H.consts, H.ell);
      const int one = single_slot;
      for (int c0 = 0; c0 < nb; c0 += 4 * PT_GROUP)
        select_sum_planes(P->T, H.consts, pv.planes + (size_t)(c0 / PT_GROUP) * gbytes,
                          cplanes.as<int8_t>(nq == 1 ? (size_t)one * cpstride() : 0), (long)cpstride(),
                          nq == 1 ? nullptr : qslot, nq, std::min(4 * PT_GROUP, nb - c0), H.ell,
                          Sx + (size_t)c0 * nq * 2 * L * n, s);
    } else if (nq == 1) {
      select_sum(P->T, H.consts, chat.as<uint64_t>((size_t)single_slot * cstride()), pv.p, pv.gs, pv.bfirst,
                 H.ell, nb, Sx, (long)(2 * L * n), s);
    } else
      select_sum_multi(P->T, H.consts, chat.as<uint64_t>(), (long)cstride(), qslot, nq, pv.p, pv.gs, pv.bfirst,
                       H.ell, nb, Sx, s);
    if (a) {
      (void)hipEventRecord(b, s);
      const uint64_t bytes =
          8ull * n * L * ((uint64_t)nb * H.ell + 2ull * H.ell * nq + 2ull * nb * nq);
      timer->pending.push_back({a, b, 0, bytes});
    }
  }

  // Select-and-sum of one tile: batches [b0, b0 + nb) of nq active queries (slots qslot[0..nq), or
  // single_slot when nq == 1) into Sout [nb * nq][2][L][N]; plaintexts from the cache (pv) or
  // generated.
  int produce_s(const uint16_t* cw, int b0, int nb, int nq, const int* qslot, int single_slot,
                const PtView& pv, uint64_t* Sout, hipStream_t s) {
    const HostParams& H = P->H;
    const size_t n = H.n, L = H.L;
    if (pv.p || (pv.planes && planes_on)) {
      timed_select_sum(pv, nb, nq, qslot, single_slot, Sout, s);
      return 0;
    }
    // a tile the resident plaintexts do not cover needs the generation buffers of setup()
    if (GB <= 0 || !gen_poly.p || !gen_p.p)
      return fail(PEPSI_E_ARG, "batches [%d, %d) are neither resident nor generable by this workspace", b0, b0 + nb);
    for (int g0 = 0; g0 < nb; g0 += GB) {
      const int g = std::min(GB, nb - g0);
      encode_server_planes(P->T, H.logn, cw, H.h, H.ell, b0 + g0, g, gen_poly.as<uint32_t>(), s);
      PtLayout pl;
      pl.ell = H.ell;
      pl.gs = GB;
      ntt_forward_plaintexts(P->T, H.logn, gen_poly.as<uint32_t>(), gen_p.as<uint64_t>(), g, (int)L, pl, s);
      PtView gv;
      gv.p = gen_p.as<uint64_t>();
      gv.gs = GB;
      timed_select_sum(gv, g, nq, qslot, single_slot, Sout + (size_t)g0 * nq * 2 * L * n, s);
    }
    return 0;
  }

  // The product tree of one tile from its select-and-sum outputs Sin, and the accumulation.
  void consume_s(uint64_t* Sin, int b0, int nb, int nq, const int* qslot, int single_slot, hipStream_t s) {
    const HostParams& H = P->H;
    const size_t n = H.n, L = H.L, K = H.K;
    const int npairs = nb * nq;
    const int* acc_slot = nq == 1 ? nullptr : qslot;
    const size_t acc_q = nq == 1 ? (size_t)single_slot : 0;
    uint64_t* acc_base = acc.as<uint64_t>(acc_q * ctw());
    const uint64_t* vtile = vhat ? vhat + (size_t)b0 * L * n : nullptr;
    if (levels == 0) {                                           // h = 1: e = S
      if (vtile)
        value_accumulate(P->T, H.consts, Sin, (long)(2 * L * n), vtile, nb, nq, acc_slot, acc_base, (long)ctw(), s);
      else
        accumulate(P->T, H.consts, Sin, (long)(2 * L * n), nb, nq, 2 * (int)L, acc_slot, acc_base, (long)ctw(), s);
      return;
    }
    uint64_t* Sq = sq.as<uint64_t>();
    if (Sin != Sq) {
      if (H.h % 2) {            // a raw factor reaches a later level: its tensor jobs read sq
        copy_words(Sq, Sin, (size_t)npairs * 2 * L * n, s);
      } else {
        Sq = Sin;
      }
    }
    tinv(Sq, scoef.as<uint64_t>(), npairs * 2 * (int)L, (int)L, 0, s);
    timed_rns(5, (uint64_t)npairs * 2 * n * ext_products(), s, [&] {
      ext_q_to_b(P->T, H.consts, scoef.as<uint64_t>(), sb.as<uint64_t>(), (long)(K * n), npairs * 2,
                 P->fallback.as<uint32_t>(), s);
    });
    tfwd(sb.p, sbh.p, npairs * 2 * (int)K, (int)K, (int)L, s);
    factor_constants(P->T, H.consts, scoef.as<uint64_t>(), npairs, H.h, alpha.as<uint64_t>(), pconst.as<uint64_t>(),
                     P->fallback.as<uint32_t>(), s);
    // the key of a single active query: shift the key base to its slot
    const int* rslot = nq == 1 ? nullptr : qslot;
    const int key_slot = nq == 1 ? single_slot : 0;
    for (int lv = 0; lv < levels; ++lv) {
      int units, jobs_per_unit, units_per_pair;
      if (lv == 0) {
        first_level(Sq, npairs, s);
        units = npairs, jobs_per_unit = H.h / 2, units_per_pair = 1;
      } else {
        const TensorJob* jl = jobs.as<TensorJob>() + job_off_na[nq][lv];
        units = npairs * jobs_at[lv], jobs_per_unit = 1, units_per_pair = jobs_at[lv];
        later_level(jl, units, s);
      }
      if (lv + 1 < levels) {
        relin_stage(units, jobs_per_unit, units_per_pair, nq, rslot, rq[lv].as<uint64_t>(), rb[lv].as<uint64_t>(),
                    s, key_slot);
      } else if (vtile) {
        // server values (Alg. 4 / 5): each pair's equality ciphertext is needed on its own,
        // relinearised, to be multiplied by its batch's value plaintext
        relin_stage(units, jobs_per_unit, units_per_pair, nq, rslot, e.as<uint64_t>(), nullptr, s, key_slot);
        value_accumulate(P->T, H.consts, e.as<uint64_t>(), (long)(2 * L * n), vtile, nb, nq, acc_slot, acc_base,
                         (long)ctw(), s);
      } else {
        // The last level's relinearisation is linear in (c01, D), so both are summed over the
        // batches (coefficient form, one entry per pair) and the key is applied once per query.
        accumulate(P->T, H.consts, c01.as<uint64_t>(), (long)(2 * L * n), nb, nq, 2 * (int)L, acc_slot, acc_base,
                   (long)ctw(), s);
        accumulate_digits(P->T, H.consts, c2.as<uint64_t>(), (long)(L * n), nb, nq, acc_slot,
                          accD.as<uint64_t>(acc_q * dtw()), (long)dtw(), s);
      }
    }
  }

  // One tile on one stream.
  int run_tile(const uint16_t* cw, int b0, int nb, int nq, const int* qslot, int single_slot,
               const PtView& pv, hipStream_t s) {
    int rc = produce_s(cw, b0, nb, nq, qslot, single_slot, pv, sq.as<uint64_t>(), s);
    if (rc) return rc;
    consume_s(sq.as<uint64_t>(), b0, nb, nq, qslot, single_slot, s);
    return 0;
  }

  // out = coefficient form of query q's sum, optionally times (h!)^-1 plus Delta [encode(mask)]_t
  void finish(int q, bool finalize, const uint32_t* mask, uint64_t* out, hipStream_t s) {
    const HostParams& H = P->H;
    const int L = H.L;
    uint64_t* a = acc.as<uint64_t>(q * ctw());
    if (levels > 0 && !vhat) {
      // a = NTT(sum of c01) + sum_i NTT(sum of D_i) (.) rlk_i
      uint64_t* dq = accD.as<uint64_t>(q * dtw());
      tfwd(a, a, 2 * L, L, 0, s);
      tfwd(dq, dq, L * L, L, 0, s);
      relin_inner(P->T, H.consts, a, dq, rlkhat.as<uint64_t>((size_t)q * rstride()), (long)rstride(), nullptr, 1, 1,
                  1, a, 1, s);
    }
    if (finalize) {
      uint64_t hf = 1;
      for (int r = 2; r <= H.h; ++r) hf = hf * r % PEPSI_T;
      const uint64_t k = powm(hf, PEPSI_T - 2, PEPSI_T);       // (h!)^-1 mod t
      const int64_t kc = k <= (PEPSI_T - 1) / 2 ? (int64_t)k : (int64_t)k - PEPSI_T;
      uint64_t kq[PEPSI_MAXL];
      for (int l = 0; l < L; ++l) kq[l] = kc >= 0 ? (uint64_t)kc : H.primes[l] - (uint64_t)(-kc);
      scale_const(P->T, H.consts, a, kq, s);
    }
    tinv(a, out, 2 * L, L, 0, s);
    if (finalize && mask) {
      uint32_t* m = reinterpret_cast<uint32_t*>(e.p);            // e is free after the tiles
      encode_slots(P->T, H.logn, mask, m, 1, s);
      add_plain_poly(P->T, H.consts, out, m, s);
    }
  }

  // Plaintexts of tile [b0, b0 + nb): the cache when it covers the tile, else generated.
  // With digit planes of the first plane_batches batches (groups of 16, group_bytes each), a
  // tile that starts a group and lies inside them also gets its planes.
  static PtView cached_tile(const uint64_t* cache, uint32_t cached, uint32_t b0, int nb,
                            const int8_t* planes = nullptr, size_t group_bytes = 0, uint32_t plane_batches = 0) {
    PtView v;
    if (cache && b0 + (uint32_t)nb <= cached) {
      v.p = cache;
      v.gs = cache_group(cached);
      v.bfirst = (int)b0;
    }
    if (planes && b0 % PT_GROUP == 0 && b0 + (uint32_t)nb <= plane_batches)
      v.planes = planes + (size_t)(b0 / PT_GROUP) * group_bytes;
    return v;
  }

  // The whole computation for nq queries in slots 0..nq-1 over batches [begin, stop).  (Running
  // the HBM-bound select-and-sum of the next tile on a second stream beside the product tree
  // was measured slower: the select-and-sum needs nearly full occupancy to cover HBM latency.)
  // Run mode: the select-and-sum of many tiles in one matrix-core launch over whole 16-batch
  // groups of digit planes (each query's request planes read once per run), into a buffer of
  // run_cap x Qmax pairs; the tiles' product trees then read their slices of it.  Enabled when
  // the planes are on, the code length fits the kernel's LDS staging, and at least one tile's
  // outputs fit beside a 4 GiB reserve; off otherwise (the tiles then run one by one).
  int enable_run(uint32_t max_batches) {
    run_cap = 0;
    if (!planes_on || plane_kblocks(P->H.ell) > PL_RUN_KBS) return 0;
    const size_t per_batch = (size_t)Qmax * ctw() * 8;
    uint32_t want = (max_batches + PT_GROUP - 1) / PT_GROUP * PT_GROUP;
    const uint32_t unit = TBq % PT_GROUP == 0 ? (uint32_t)TBq : (uint32_t)PT_GROUP * TBq;
    want = (want + unit - 1) / unit * unit;
    if (sall.cap < (size_t)want * per_batch) {
      size_t free_b = 0, total_b = 0;
      if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail(PEPSI_E_DEVICE, "hipMemGetInfo failed");
      const size_t reserve = (size_t)4 << 30, have = free_b > reserve ? free_b - reserve : 0;
      const uint32_t fit = (uint32_t)std::min<size_t>(have / per_batch + sall.cap / per_batch, want);
      want = fit / unit * unit;
      if (want < (uint32_t)TBq) return 0;
      sall.release();
      int rc = sall.ensure((size_t)want * per_batch);
      if (rc) return rc;
    }
    run_cap = want;
    return 0;
  }

  int run(const uint16_t* cw, const uint64_t* cache, uint32_t cached, uint32_t begin, uint32_t stop, int nq,
          const uint64_t* const* cts, const uint64_t* const* rlk, hipStream_t s, const int8_t* planes = nullptr,
          size_t group_bytes = 0, uint32_t plane_batches = 0) {
    const HostParams& H = P->H;
    for (int q = 0; q < nq; ++q) admit(q, cts[q], rlk[q], s);
    uint32_t b0 = begin;
    while (b0 < stop) {
      if (run_cap > 0 && planes && planes_on && b0 % PT_GROUP == 0 && b0 < plane_batches) {
        const uint32_t r1 = std::min<uint32_t>(std::min<uint32_t>(stop, plane_batches), b0 + run_cap);
        const int nb = (int)(r1 - b0), ng = (nb + PT_GROUP - 1) / PT_GROUP;
        hipEvent_t a = nullptr, b = nullptr;
        if (timer && timer->on) { a = timer->get(); b = timer->get(); (void)hipEventRecord(a, s); }
        select_sum_planes_run(P->T, H.consts, planes + (size_t)(b0 / PT_GROUP) * group_bytes, ng, cplanes.as<int8_t>(),
                              (long)cpstride(), nullptr, nq, nb, H.ell, sall.as<uint64_t>(), s);
        if (a) {
          (void)hipEventRecord(b, s);
          const uint64_t bytes = 8ull * H.n * H.L * ((uint64_t)nb * H.ell + 2ull * H.ell * nq + 2ull * nb * nq);
          timer->pending.push_back({a, b, 0, bytes});
        }
        for (uint32_t t0 = b0; t0 < r1; t0 += TBq) {
          const int nbt = (int)std::min<uint32_t>(TBq, r1 - t0);
          consume_s(sall.as<uint64_t>((size_t)(t0 - b0) * nq * ctw()), (int)t0, nbt, nq, nullptr, 0, s);
        }
        b0 = r1;
        continue;
      }
      const int nb = (int)std::min<uint32_t>(TBq, stop - b0);
      const int rc = run_tile(cw, (int)b0, nb, nq, nullptr, 0,
                              cached_tile(cache, cached, b0, nb, planes, group_bytes, plane_batches), s);
      if (rc) return rc;
      b0 += TBq;
    }
    return 0;
  }
};

}  // namespace

// Engine device memory: per (batch, query) pair of tile buffers, and per query slot (request,
// key and sums in NTT form).
static size_t engine_pair_bytes(const HostParams& H) {
  const size_t n = H.n, L = H.L, K = H.K, Pn = L + K;
  const size_t jobs0 = (size_t)(H.h / 2 > 0 ? H.h / 2 : 1);
  return 8 * n * (2 * L * 3 + 4 * K + jobs0 * (3 * Pn + 5 * L + L * L + 2 * L + 2 * L + 2 * K));
}
static size_t engine_slot_bytes(const HostParams& H) {
  const size_t n = H.n, L = H.L;
  return 8 * ((size_t)H.ell * 2 * L * n + L * 2 * L * n + 2 * L * n);
}

// ------------------------------------------------------------------ batched schedules
namespace {
// Launch sequences of batched evaluations captured into HIP graphs, keyed by the query count and
// the caller's buffers (the kernels' arguments); the engine's own buffers are fixed until its
// workspace is set up again, which clears the cache.
struct GraphCache {
  struct Entry {
    std::vector<uintptr_t> key;
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
  };
  static constexpr size_t kMax = 4;
  std::vector<Entry> entries;        // least recently used first
  hipStream_t cap = nullptr;         // capture stream (the caller's may be the null stream)
  void clear() {
    for (auto& x : entries) {
      if (x.e) (void)hipGraphExecDestroy(x.e);
      if (x.g) (void)hipGraphDestroy(x.g);
    }
    entries.clear();
  }
  Entry* find(const std::vector<uintptr_t>& key) {
    for (size_t i = 0; i < entries.size(); ++i)
      if (entries[i].key == key) {
        std::rotate(entries.begin() + i, entries.begin() + i + 1, entries.end());
        return &entries.back();
      }
    return nullptr;
  }
  ~GraphCache() {
    clear();
    if (cap) (void)hipStreamDestroy(cap);
  }
};

// Schedules measured by autotune.py on MI355X: {log_n, L, ell, h, nq_max, tile_batches,
// select_kernel, graph, run, ms_per_query}.
struct TunedEntry { int logn, L, ell, h, nq_max, tile, kernel, graph, run; double ms; };
const TunedEntry kTuned[] = {
#include "schedule_table.inc"
    {0, 0, 0, 0, 0, 0, 0, 0, 0, 0.0}};

const TunedEntry* tuned_entry(const HostParams& H, uint32_t nq) {
  const TunedEntry* best = nullptr;
  for (const TunedEntry& t : kTuned)
    if (t.logn == H.logn && t.L == H.L && t.ell == H.ell && t.h == H.h && (uint32_t)t.nq_max >= nq &&
        (!best || t.nq_max < best->nq_max))
      best = &t;
  return best;
}
}  // namespace

// ------------------------------------------------------------------ server
struct pepsi_server {
  pepsi_params* P = nullptr;
  EventTimer timer;
  uint32_t max_load = 0;
  DevBuf cw;            // [mu][N][h] uint16
  DevBuf cache;         // plaintext store of the cached batches (layout at PtLayout)
  bool cached = false;
  uint32_t cached_batches = 0;
  DevBuf planes;        // digit planes of the cached 16-batch groups (matrix-core select-and-sum)
  uint32_t plane_groups = 0;
  uint32_t plane_batches = 0;  // batches covered by the planes (the first ones)
  size_t plane_group_bytes = 0;
  bool planes_only = false;    // plaintexts kept only as digit planes
  const int8_t* planes_p() const { return plane_groups ? planes.as<int8_t>() : nullptr; }
  // On-the-fly generation: the single-query engine needs it unless the NTT-form cache covers
  // every batch holding items (its ranges may start anywhere); the many-query engines walk
  // group-aligned tiles, which the planes cover too.
  bool need_gen_single() const { return cached_batches < max_load; }
  bool need_gen_multi() const { return cached_batches < max_load && plane_batches < max_load; }
  Engine eng;            // one query at a time (plain path)
  bool ready = false;
  Engine beng;           // many queries per launch (batched path)
  int bqmax = 0;
  pepsi_schedule bsched{};     // schedule the batched workspace was set up for
  pepsi_schedule forced{};     // caller's schedule (fields 0: automatic)
  GraphCache graphs;           // captured batched evaluations
  DevBuf vhat;           // server values (Alg. 4 / 5): [max_load][L][N] plaintexts, NTT form
  bool valued = false;
  const uint64_t* values_hat() const { return valued ? vhat.as<uint64_t>() : nullptr; }
};

extern "C" int pepsi_server_create(const pepsi_params* Pc, const uint32_t* items, uint64_t n,
                                   uint32_t flags, void* stream, pepsi_server** out) {
  return pepsi_server_create_with_values(Pc, items, nullptr, n, flags, stream, out);
}

extern "C" int pepsi_server_create_with_values(const pepsi_params* Pc, const uint32_t* items,
                                               const uint32_t* values, uint64_t n, uint32_t flags, void* stream,
                                               pepsi_server** out) {
  return pepsi_server_create_ex(Pc, items, values, n, flags, 0, stream, out);
}

static int server_create_impl(const pepsi_params* Pc, const uint64_t* items, const uint32_t* values, uint64_t n,
                              uint32_t flags, uint32_t max_cached, void* stream, pepsi_server** out);

extern "C" int pepsi_server_create_ex(const pepsi_params* Pc, const uint32_t* items, const uint32_t* values,
                                      uint64_t n, uint32_t flags, uint32_t max_cached, void* stream,
                                      pepsi_server** out) {
  if (!Pc || (!items && n) || !out) return fail(PEPSI_E_ARG, "null argument");
  std::vector<uint64_t> wide(items, items + n);
  return server_create_impl(Pc, wide.data(), values, n, flags, max_cached, stream, out);
}

extern "C" int pepsi_server_create64(const pepsi_params* Pc, const uint64_t* items, const uint32_t* values,
                                     uint64_t n, uint32_t flags, uint32_t max_cached, void* stream,
                                     pepsi_server** out) {
  if (!Pc || (!items && n) || !out) return fail(PEPSI_E_ARG, "null argument");
  return server_create_impl(Pc, items, values, n, flags, max_cached, stream, out);
}

static int server_create_impl(const pepsi_params* Pc, const uint64_t* items, const uint32_t* values, uint64_t n,
                              uint32_t flags, uint32_t max_cached, void* stream, pepsi_server** out) {
  pepsi_params* P = const_cast<pepsi_params*>(Pc);
  if (!P || (!items && n) || !out) return fail(PEPSI_E_ARG, "null argument");
  *out = nullptr;
  if (flags & ~(PEPSI_SERVER_CACHE_PLAINTEXTS | PEPSI_SERVER_PLANES_ONLY)) return fail(PEPSI_E_ARG, "unknown flags");
  if ((flags & PEPSI_SERVER_PLANES_ONLY) && !(flags & PEPSI_SERVER_CACHE_PLAINTEXTS))
    return fail(PEPSI_E_ARG, "PEPSI_SERVER_PLANES_ONLY needs PEPSI_SERVER_CACHE_PLAINTEXTS");
  const HostParams& H = P->H;
  {
    std::unordered_set<uint64_t> seen;
    seen.reserve(n * 2);
    for (uint64_t i = 0; i < n; ++i) {
      if (H.item_bits < 64 && (items[i] >> H.item_bits)) return fail(PEPSI_E_RANGE, "server item out of range");
      if (!seen.insert(items[i]).second) return fail(PEPSI_E_RANGE, "duplicate server item");
      if (values && values[i] >= PEPSI_T) return fail(PEPSI_E_RANGE, "server value not below t");
    }
  }
  std::vector<uint64_t> table;
  std::vector<uint32_t> index;
  std::vector<uint8_t> valid;
  uint32_t max_load = 0;
  if (simple_hash(items, n, H.n, H.hash_seed, H.n_hash, H.mu, &table, &valid, &max_load,
                  values ? &index : nullptr, H.pbh ? H.item_bits : 0))
    return fail(PEPSI_E_BIN_OVERFLOW, "a server bin exceeds mu = %d", H.mu);
  std::vector<uint16_t> cw((size_t)H.mu * H.n * H.h, 0xFFFF);
  CwEncoder enc(H.ell, H.h);
  for (size_t i = 0; i < (size_t)H.mu * H.n; ++i)
    if (valid[i]) enc.encode(table[i], &cw[i * H.h]);
  pepsi_server* sv = new pepsi_server();
  sv->P = P;
  sv->max_load = max_load;
  int rc = sv->cw.ensure(cw.size() * 2);
  if (rc) { delete sv; return rc; }
  if (hipMemcpy(sv->cw.p, cw.data(), cw.size() * 2, hipMemcpyHostToDevice) != hipSuccess) {
    delete sv;
    return fail(PEPSI_E_DEVICE, "codeword upload failed");
  }
  if (values && max_load > 0) {
    // val_s[i'] for the batches that hold real items: slot k = value of the item at (i', k)
    // (0 for dummies), batch-encoded, lifted and transformed once into NTT form
    std::vector<uint32_t> vt((size_t)max_load * H.n, 0);
    for (size_t i = 0; i < vt.size(); ++i)
      if (valid[i]) vt[i] = values[index[i]];
    DevBuf raw, poly;
    if ((rc = raw.ensure(vt.size() * 4)) || (rc = poly.ensure(vt.size() * 4)) ||
        (rc = sv->vhat.ensure(vt.size() * H.L * 8))) {
      delete sv;
      return rc;
    }
    hipStream_t s = S(stream);
    if (hipMemcpyAsync(raw.p, vt.data(), vt.size() * 4, hipMemcpyHostToDevice, s) != hipSuccess) {
      delete sv;
      return fail(PEPSI_E_DEVICE, "value upload failed");
    }
    encode_slots(P->T, H.logn, raw.as<uint32_t>(), poly.as<uint32_t>(), (int)max_load, s);
    ntt_forward(P->T, H.logn, poly.p, LOAD_LIFT_T, sv->vhat.p, STORE_U64, (int)max_load * H.L, H.L, 0, s);
    if (hipStreamSynchronize(s) != hipSuccess) { delete sv; return fail(PEPSI_E_DEVICE, "value encoding failed"); }
    sv->valued = true;
  }
  if ((flags & PEPSI_SERVER_PLANES_ONLY) && max_load > 0 && planes_supported(H.ell)) {
    // digit planes only, as many 16-batch groups as fit beside the working reserve (and the
    // one-group staging store they are generated in)
    const size_t gb = plaintext_plane_group_bytes(H.consts, H.ell);
    const size_t stage = (size_t)PT_GROUP * H.ell * H.L * H.n * 8;
    const size_t reserve = (size_t)48 << 30;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { delete sv; return fail(PEPSI_E_DEVICE, "hipMemGetInfo failed"); }
    const uint32_t all = (max_load + PT_GROUP - 1) / PT_GROUP;
    uint32_t groups = (uint32_t)std::min<size_t>(free_b > reserve + stage ? (free_b - reserve - stage) / gb : 0, all);
    if (max_cached > 0 && max_cached < max_load) groups = std::min(groups, max_cached / PT_GROUP);
    if (groups > 0) {
      DevBuf stg, poly;
      const int G8 = 8;
      if ((rc = sv->planes.ensure(gb * groups)) || (rc = stg.ensure(stage)) ||
          (rc = poly.ensure((size_t)G8 * H.ell * H.n * 4))) {
        delete sv;
        return rc;
      }
      hipStream_t s = S(stream);
      for (uint32_t G = 0; G < groups; ++G) {
        const uint32_t gend = std::min<uint32_t>((G + 1) * PT_GROUP, max_load);
        for (uint32_t b0 = G * PT_GROUP; b0 < gend; b0 += G8) {
          const int g = (int)std::min<uint32_t>(G8, gend - b0);
          encode_server_planes(P->T, H.logn, sv->cw.as<uint16_t>(), H.h, H.ell, (int)b0, g, poly.as<uint32_t>(), s);
          PtLayout pl;
          pl.ell = H.ell;
          pl.gs = PT_GROUP;
          pl.bbase = (int)(b0 - G * PT_GROUP);
          ntt_forward_plaintexts(P->T, H.logn, poly.as<uint32_t>(), stg.as<uint64_t>(), g, H.L, pl, s);
        }
        plaintext_planes(P->T, H.consts, stg.as<uint64_t>(), PT_GROUP, 0, H.ell, sv->planes.as<int8_t>((size_t)G * gb),
                         s);
      }
      if (hipStreamSynchronize(s) != hipSuccess) { delete sv; return fail(PEPSI_E_DEVICE, "plane build failed"); }
      sv->plane_groups = groups;
      sv->plane_batches = std::min<uint32_t>(groups * PT_GROUP, max_load);
      sv->plane_group_bytes = gb;
      sv->planes_only = true;
    }
  } else if ((flags & PEPSI_SERVER_CACHE_PLAINTEXTS) && max_load > 0) {
    // as many batches as fit beside a working reserve, in whole 16-batch tiles unless all fit
    const size_t per = (size_t)H.ell * H.L * H.n;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { delete sv; return fail(PEPSI_E_DEVICE, "hipMemGetInfo failed"); }
    const size_t reserve = (size_t)48 << 30;
    size_t fit = free_b > reserve ? (free_b - reserve) / (per * 8) : 0;
    uint32_t nc = (uint32_t)std::min<size_t>(fit, max_load);
    if (max_cached > 0) nc = std::min(nc, max_cached);
    if (nc < max_load) nc -= nc % PT_GROUP;
    if (nc > 0) {
      const int gs = Engine::cache_group(nc);
      const size_t alloc_b = (nc + gs - 1) / gs * gs;
      if ((rc = sv->cache.ensure(per * alloc_b * 8))) { delete sv; return rc; }
      DevBuf poly;
      const int G = 8;
      if ((rc = poly.ensure((size_t)G * H.ell * H.n * 4))) { delete sv; return rc; }
      hipStream_t s = S(stream);
      for (uint32_t b0 = 0; b0 < nc; b0 += G) {
        const int g = (int)std::min<uint32_t>(G, nc - b0);
        encode_server_planes(P->T, H.logn, sv->cw.as<uint16_t>(), H.h, H.ell, (int)b0, g, poly.as<uint32_t>(), s);
        PtLayout pl;
        pl.ell = H.ell;
        pl.gs = gs;
        pl.bbase = (int)b0;
        ntt_forward_plaintexts(P->T, H.logn, poly.as<uint32_t>(), sv->cache.as<uint64_t>(), g, H.L, pl, s);
      }
      if (hipStreamSynchronize(s) != hipSuccess) { poly.release(); delete sv; return fail(PEPSI_E_DEVICE, "cache build failed"); }
      poly.release();
      sv->cached = true;
      sv->cached_batches = nc;
      // digit planes of the cached groups for the batched path, when they fit beside the reserve
      const uint32_t groups = (nc + PT_GROUP - 1) / PT_GROUP;
      const size_t gb = plaintext_plane_group_bytes(H.consts, H.ell);
      if (gs == PT_GROUP && planes_supported(H.ell)) {
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) { delete sv; return fail(PEPSI_E_DEVICE, "hipMemGetInfo failed"); }
        if (free_b > reserve && (free_b - reserve) / gb >= groups) {
          if ((rc = sv->planes.ensure(gb * groups))) { delete sv; return rc; }
          for (uint32_t G = 0; G < groups; ++G)
            plaintext_planes(P->T, H.consts, sv->cache.as<uint64_t>(), gs, (int)G, H.ell,
                             sv->planes.as<int8_t>((size_t)G * gb), s);
          if (hipStreamSynchronize(s) != hipSuccess) { delete sv; return fail(PEPSI_E_DEVICE, "plane build failed"); }
          sv->plane_groups = groups;
          sv->plane_batches = nc;
          sv->plane_group_bytes = gb;
        }
      }
    }
  }
  *out = sv;
  return PEPSI_OK;
}

extern "C" int pepsi_server_get_info(const pepsi_server* sv, pepsi_server_info* o) {
  if (!sv || !o) return fail(PEPSI_E_ARG, "null argument");
  memset(o, 0, sizeof(*o));
  o->mu = sv->P->H.mu;
  o->max_load = sv->max_load;
  o->cached = sv->cached ? 1 : 0;
  o->cached_batches = sv->cached_batches;
  o->device_bytes = sv->cw.cap + sv->cache.cap + sv->vhat.cap + sv->planes.cap;
  o->plane_groups = sv->plane_groups;
  return PEPSI_OK;
}

extern "C" int pepsi_server_codewords(const pepsi_server* sv, uint16_t* out) {
  if (!sv || !out) return fail(PEPSI_E_ARG, "null argument");
  const HostParams& H = sv->P->H;
  HIPCHK(hipMemcpy(out, sv->cw.p, (size_t)H.mu * H.n * H.h * 2, hipMemcpyDeviceToHost));
  return PEPSI_OK;
}

extern "C" void pepsi_server_destroy(pepsi_server* sv) {
  if (!sv) return;
  (void)hipDeviceSynchronize();
  sv->graphs.clear();
  sv->cw.release();
  sv->cache.release();
  sv->vhat.release();
  sv->planes.release();
  delete sv;
}

extern "C" int pepsi_server_eval_range(pepsi_server* sv, const uint64_t* cts, const uint64_t* rlk,
                                       uint32_t begin, uint32_t end, uint32_t finalize,
                                       const uint32_t* mask, uint64_t* out, void* stream) {
  if (!sv || !cts || !rlk || !out) return fail(PEPSI_E_ARG, "null argument");
  const HostParams& H = sv->P->H;
  if (begin > end || end > (uint32_t)H.mu) return fail(PEPSI_E_ARG, "bad batch range");
  hipStream_t s = S(stream);
  if (!sv->ready) {
    const int tb = std::min<int>(512, std::max<int>(1, (int)sv->max_load));
    int rc = sv->eng.setup(sv->P, tb, 1, sv->need_gen_single(), sv->values_hat());
    if (!rc && sv->planes_only) rc = sv->eng.enable_planes(true);
    if (rc) return rc;
    sv->eng.timer = &sv->timer;
    sv->ready = true;
  }
  Engine& E = sv->eng;
  hipEvent_t ea = nullptr, eb = nullptr;
  if (sv->timer.on) { ea = sv->timer.get(); eb = sv->timer.get(); (void)hipEventRecord(ea, s); }
  // batches at or above the fullest bin hold only dummies: their equality ciphertext is (0, 0)
  const uint32_t stop = std::min(end, sv->max_load);
  const uint64_t* c1[1] = {cts};
  const uint64_t* r1[1] = {rlk};
  int rc = E.run(sv->cw.as<uint16_t>(), sv->cached ? sv->cache.as<uint64_t>() : nullptr, sv->cached_batches, begin,
                 std::max(begin, stop), 1, c1, r1, s, sv->planes_only ? sv->planes_p() : nullptr,
                 sv->plane_group_bytes, sv->plane_batches);
  if (rc) return rc;
  E.finish(0, finalize != 0, mask, out, s);
  if (ea) {
    (void)hipEventRecord(eb, s);
    sv->timer.pending.push_back({ea, eb, 1, 0});
  }
  HIPCHK(hipGetLastError());
  return PEPSI_OK;
}

extern "C" int pepsi_server_eval(pepsi_server* sv, const uint64_t* cts, const uint64_t* rlk,
                                 const uint32_t* mask, uint64_t* out, void* stream) {
  if (!sv) return fail(PEPSI_E_ARG, "null argument");
  return pepsi_server_eval_range(sv, cts, rlk, 0, sv->P->H.mu, 1, mask, out, stream);
}

// The schedule of a batched evaluation of nq queries (see pepsi_schedule): the caller's fields,
// then the tuned table, then the rule.  The tile size is the one requested; eval_batch falls back
// to 16 batches when its workspace does not fit.
static pepsi_schedule resolve_schedule(const pepsi_server* sv, uint32_t nq) {
  const HostParams& H = sv->P->H;
  pepsi_schedule r{};
  r.source = PEPSI_SCHEDULE_DEFAULT;
  if (const TunedEntry* t = tuned_entry(H, nq)) {
    r.tile_batches = (uint32_t)t->tile;
    r.select_kernel = (uint32_t)t->kernel;
    r.graph = (uint32_t)t->graph;
    r.run = (uint32_t)t->run;
    r.tuned_ms_per_query = t->ms;
    r.source = PEPSI_SCHEDULE_TUNED;
  }
  const pepsi_schedule& f = sv->forced;
  if (f.tile_batches || f.select_kernel || f.graph || f.run) r.source = PEPSI_SCHEDULE_CALLER;
  if (f.tile_batches) r.tile_batches = f.tile_batches;
  if (f.select_kernel) r.select_kernel = f.select_kernel;
  if (f.graph) r.graph = f.graph;
  if (!r.select_kernel) r.select_kernel = sv->plane_groups > 0 ? PEPSI_SELECT_PLANES : PEPSI_SELECT_VALU;
  if (sv->plane_groups == 0) r.select_kernel = PEPSI_SELECT_VALU;      // nothing to contract on the matrix cores
  if (sv->planes_only) r.select_kernel = PEPSI_SELECT_PLANES;         // the plaintexts exist only as planes
  if (!r.graph) r.graph = PEPSI_GRAPH_ON;
  if (f.run) r.run = f.run;
  if (!r.run) r.run = PEPSI_RUN_ON;
  if (r.select_kernel != PEPSI_SELECT_PLANES) r.run = PEPSI_RUN_OFF;        // runs are a matrix-core form
  if (!r.tile_batches) r.tile_batches = (r.select_kernel == PEPSI_SELECT_PLANES && nq <= 64) ? 64 : 16;
  return r;
}

extern "C" int pepsi_server_set_schedule(pepsi_server* sv, const pepsi_schedule* sch) {
  if (!sv) return fail(PEPSI_E_ARG, "null argument");
  pepsi_schedule f{};
  if (sch) {
    if (sch->tile_batches && sch->tile_batches != 16 && sch->tile_batches != 32 && sch->tile_batches != 64)
      return fail(PEPSI_E_ARG, "tile_batches must be 0, 16, 32 or 64");
    if (sch->select_kernel > PEPSI_SELECT_VALU) return fail(PEPSI_E_ARG, "unknown select kernel");
    if (sch->graph > PEPSI_GRAPH_OFF) return fail(PEPSI_E_ARG, "unknown graph mode");
    if (sch->run > PEPSI_RUN_OFF) return fail(PEPSI_E_ARG, "unknown run mode");
    if (sch->select_kernel == PEPSI_SELECT_VALU && sv->planes_only)
      return fail(PEPSI_E_ARG, "the server keeps its plaintexts only as digit planes");
    f.tile_batches = sch->tile_batches;
    f.select_kernel = sch->select_kernel;
    f.graph = sch->graph;
    f.run = sch->run;
  }
  sv->forced = f;
  return PEPSI_OK;
}

extern "C" int pepsi_server_get_schedule(pepsi_server* sv, uint32_t nq, pepsi_schedule* out) {
  if (!sv || !out) return fail(PEPSI_E_ARG, "null argument");
  *out = resolve_schedule(sv, nq ? nq : 1);
  return PEPSI_OK;
}

extern "C" int pepsi_server_eval_batch(pepsi_server* sv, uint32_t nq, const uint64_t* const* cts,
                                       const uint64_t* const* rlk, const uint32_t* const* masks,
                                       uint64_t* const* out, void* stream) {
  if (!sv || !cts || !rlk || !out) return fail(PEPSI_E_ARG, "null argument");
  if (nq == 0) return PEPSI_OK;
  if (nq > PEPSI_MAX_BATCH) return fail(PEPSI_E_ARG, "at most %d queries per batch", PEPSI_MAX_BATCH);
  for (uint32_t q = 0; q < nq; ++q)
    if (!cts[q] || !rlk[q] || !out[q]) return fail(PEPSI_E_ARG, "null query pointer %u", q);
  const HostParams& H = sv->P->H;
  hipStream_t s = S(stream);
  const pepsi_schedule want = resolve_schedule(sv, nq);
  const bool planes = want.select_kernel == PEPSI_SELECT_PLANES;
  if ((int)nq > sv->bqmax || want.select_kernel != sv->bsched.select_kernel ||
      want.tile_batches != sv->bsched.tile_batches || want.run != sv->bsched.run) {
    // the requested tile when its workspace fits beside an 8 GiB reserve, else 16 batches (one
    // batch group of the select-and-sum kernels)
    if (!(planes && want.run == PEPSI_RUN_ON)) sv->beng.sall.release();   // its memory goes to the tiles
    int tb = 16;
    if (want.tile_batches > 16) {
      size_t free_b = 0, total_b = 0;
      if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return fail(PEPSI_E_DEVICE, "hipMemGetInfo failed");
      free_b += sv->beng.held_bytes() - sv->beng.sall.cap;    // the workspace's own buffers are reused
      const size_t fixed = (size_t)nq * (engine_slot_bytes(H) + (planes ? request_plane_bytes(H.consts, H.ell) : 0)) +
                           ((size_t)8 << 30);
      for (int cand : {64, 32})
        if (cand <= (int)want.tile_batches && free_b > fixed + (size_t)cand * nq * engine_pair_bytes(H)) {
          tb = cand;
          break;
        }
    }
    // the workspace counts as set up only once every part of it is (a failed call leaves
    // bqmax at 0, so the next call sets it up again instead of running on a partial one)
    sv->bqmax = 0;
    sv->graphs.clear();
    const bool need_gen = planes ? sv->need_gen_multi() : sv->cached_batches < sv->max_load;
    int rc = sv->beng.setup(sv->P, std::min<int>(tb, std::max<int>(1, (int)sv->max_load)), (int)nq, need_gen,
                            sv->values_hat());
    if (rc) return rc;
    sv->beng.timer = &sv->timer;
    if (planes && (rc = sv->beng.enable_planes(sv->planes_only))) return rc;
    if (planes && want.run == PEPSI_RUN_ON && (rc = sv->beng.enable_run(std::min<uint32_t>(H.mu, sv->max_load))))
      return rc;
    sv->bsched = want;
    sv->bqmax = (int)nq;
  }
  Engine& E = sv->beng;
  const uint32_t stop = std::min<uint32_t>(H.mu, sv->max_load);
  auto run_all = [&](hipStream_t st) -> int {
    int rc = E.run(sv->cw.as<uint16_t>(), sv->cached ? sv->cache.as<uint64_t>() : nullptr, sv->cached_batches, 0,
                   stop, (int)nq, cts, rlk, st, planes ? sv->planes_p() : nullptr, sv->plane_group_bytes,
                   sv->plane_batches);
    if (rc) return rc;
    for (uint32_t q = 0; q < nq; ++q) E.finish((int)q, true, masks ? masks[q] : nullptr, out[q], st);
    return 0;
  };
  hipEvent_t ea = nullptr, eb = nullptr;
  if (sv->timer.on) { ea = sv->timer.get(); eb = sv->timer.get(); (void)hipEventRecord(ea, s); }
  if (want.graph == PEPSI_GRAPH_ON && !sv->timer.on) {
    std::vector<uintptr_t> key;
    key.reserve(1 + 4 * (size_t)nq);
    key.push_back(nq);
    for (uint32_t q = 0; q < nq; ++q) {
      key.push_back((uintptr_t)cts[q]);
      key.push_back((uintptr_t)rlk[q]);
      key.push_back((uintptr_t)(masks ? masks[q] : nullptr));
      key.push_back((uintptr_t)out[q]);
    }
    GraphCache& gc = sv->graphs;
    GraphCache::Entry* ent = gc.find(key);
    if (!ent) {
      if (!gc.cap) HIPCHK(hipStreamCreateWithFlags(&gc.cap, hipStreamNonBlocking));
      HIPCHK(hipStreamBeginCapture(gc.cap, hipStreamCaptureModeThreadLocal));
      const int rc = run_all(gc.cap);
      hipGraph_t g = nullptr;
      const hipError_t ec = hipStreamEndCapture(gc.cap, &g);
      if (rc || ec != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return rc ? rc : fail(PEPSI_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ec));
      }
      hipGraphExec_t ex = nullptr;
      if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(PEPSI_E_DEVICE, "graph instantiation failed");
      }
      if (gc.entries.size() >= GraphCache::kMax) {
        (void)hipGraphExecDestroy(gc.entries.front().e);
        (void)hipGraphDestroy(gc.entries.front().g);
        gc.entries.erase(gc.entries.begin());
      }
      gc.entries.push_back(GraphCache::Entry{std::move(key), g, ex});
      ent = &gc.entries.back();
    }
    HIPCHK(hipGraphLaunch(ent->e, s));
  } else {
    const int rc = run_all(s);
    if (rc) return rc;
  }
  if (ea) {
    (void)hipEventRecord(eb, s);
    sv->timer.pending.push_back({ea, eb, 1, 0});
  }
  HIPCHK(hipGetLastError());
  return PEPSI_OK;
}

extern "C" int pepsi_server_timing(pepsi_server* sv, int enable, int reset, pepsi_timing* out) {
  if (!sv) return fail(PEPSI_E_ARG, "null argument");
  HIPCHK(hipDeviceSynchronize());
  if (sv->timer.fold()) return fail(PEPSI_E_DEVICE, "event timing failed");
  if (out) *out = sv->timer.tot;
  if (reset) sv->timer.tot = pepsi_timing{};
  sv->timer.on = enable != 0;
  return PEPSI_OK;
}


// ------------------------------------------------------------------ serving
// Continuous batching.  The worker walks the server batches as a circular sequence of tiles of
// TBq batches; every step runs one tile for all active queries.  A request is admitted into a
// free slot at a step boundary and is finished after it has seen every tile once (it joins at
// whatever tile the cursor is on; sums mod Q do not depend on the order).  Requests beyond the
// slots wait in the queue.
namespace {
double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}
}  // namespace

extern "C" double pepsi_clock(void) { return now_s(); }

struct pepsi_serve {
  struct Req {
    uint64_t id = 0;
    const uint64_t* cts = nullptr;
    const uint64_t* rlk = nullptr;
    const uint32_t* mask = nullptr;
    uint64_t* out = nullptr;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int slot = -1, tiles = 0, done = 0;
  };
  pepsi_server* sv = nullptr;
  Engine eng;
  hipStream_t stream = nullptr;
  int slots = 0, T = 0, cursor = 0;
  uint32_t stop_b = 0;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  bool stop = false;
  int err = 0;
  std::string err_msg;
  std::deque<Req*> queue;
  std::unordered_map<uint64_t, Req*> reqs;
  std::vector<Req*> active;
  uint64_t next_id = 1, steps = 0, completed = 0;
  int* qslot_host = nullptr;           // kDepth + 1 pinned slot lists of `slots` entries
  DevBuf qslot_dev;
  size_t slot_bytes = 0;

  // Steps are enqueued ahead of the device: up to kDepth steps in flight, each ending with an
  // event; a request is done when the event of the step that enqueued its finish has completed.
  // Host bookkeeping (admissions, slot lists, completions) thus overlaps the device's work.
  static constexpr int kDepth = 2;
  struct Step {
    hipEvent_t ev = nullptr;
    std::vector<Req*> finished;
  };
  std::deque<Step> inflight;
  std::vector<hipEvent_t> ev_pool;
  int ring = 0;

  void fail_all(const char* what) {
    std::lock_guard<std::mutex> lk(mu);
    err = PEPSI_E_DEVICE;
    err_msg = what;
    cv_done.notify_all();
  }

  // Completes the requests of finished steps, oldest first; with blocking, waits for the oldest
  // one.  Returns false after a device error.
  bool retire(bool blocking) {
    while (!inflight.empty()) {
      Step& st = inflight.front();
      const hipError_t e = blocking ? hipEventSynchronize(st.ev) : hipEventQuery(st.ev);
      if (e == hipErrorNotReady) return true;
      if (e != hipSuccess) {
        fail_all("device error in a serving step");
        return false;
      }
      if (!st.finished.empty()) {
        std::lock_guard<std::mutex> lk(mu);
        const double t = now_s();
        for (Req* r : st.finished) {
          r->t_done = t;
          r->done = 1;
          ++completed;
        }
        cv_done.notify_all();
      }
      ev_pool.push_back(st.ev);
      inflight.pop_front();
      blocking = false;
    }
    return true;
  }

  void loop() {
    (void)hipSetDevice(sv->P->device);
    for (;;) {
      if (!retire(false)) return;
      std::vector<Req*> admitted;
      bool any_active = false;
      {
        std::unique_lock<std::mutex> lk(mu);
        for (Req* r : active) any_active |= r != nullptr;
        if (!any_active && queue.empty() && inflight.empty()) {
          cv.wait(lk, [&] { return stop || !queue.empty(); });
          if (stop && queue.empty()) break;
        }
        for (int s = 0; s < slots && !queue.empty(); ++s) {
          if (active[s]) continue;
          Req* r = queue.front();
          queue.pop_front();
          r->slot = s;
          r->t_admit = now_s();
          active[s] = r;
          admitted.push_back(r);
          any_active = true;
        }
      }
      if (!any_active) {                   // only completions are pending
        if (!retire(true)) return;
        continue;
      }
      if ((int)inflight.size() >= kDepth && !retire(true)) return;
      for (Req* r : admitted) eng.admit(r->slot, r->cts, r->rlk, stream);
      std::vector<int> live;
      for (int s = 0; s < slots; ++s) if (active[s]) live.push_back(s);
      const int na = (int)live.size();
      Step st;
      if (T > 0) {
        int* hb = qslot_host + (size_t)ring * slots;      // its last reader has retired
        ring = (ring + 1) % (kDepth + 1);
        for (int i = 0; i < na; ++i) hb[i] = live[i];
        if (hipMemcpyAsync(qslot_dev.p, hb, sizeof(int) * na, hipMemcpyHostToDevice, stream) != hipSuccess) {
          fail_all("slot upload failed");
          return;
        }
        const uint32_t b0 = (uint32_t)cursor * eng.TBq;
        const int nb = (int)std::min<uint32_t>(eng.TBq, stop_b - b0);
        if (eng.run_tile(sv->cw.as<uint16_t>(), (int)b0, nb, na, qslot_dev.as<int>(), live[0],
                         Engine::cached_tile(sv->cached ? sv->cache.as<uint64_t>() : nullptr, sv->cached_batches,
                                             b0, nb, sv->planes_p(), sv->plane_group_bytes, sv->plane_batches),
                         stream)) {
          fail_all(g_err.c_str());
          return;
        }
        cursor = (cursor + 1) % T;
        ++steps;
      }
      for (int s : live) {
        Req* r = active[s];
        if (++r->tiles >= T) {
          eng.finish(s, true, r->mask, r->out, stream);
          st.finished.push_back(r);
          std::lock_guard<std::mutex> lk(mu);
          active[s] = nullptr;                           // the slot takes a new request at once
        }
      }
      if (ev_pool.empty()) {
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
          fail_all("event creation failed");
          return;
        }
        ev_pool.push_back(e);
      }
      st.ev = ev_pool.back();
      ev_pool.pop_back();
      if (hipEventRecord(st.ev, stream) != hipSuccess) {
        fail_all("event record failed");
        return;
      }
      inflight.push_back(std::move(st));
    }
    (void)retire(true);
    while (!inflight.empty())
      if (!retire(true)) return;
  }
};

extern "C" int pepsi_serve_create(pepsi_server* sv, uint32_t max_active, uint64_t hbm_budget, pepsi_serve** out) {
  if (!sv || !out) return fail(PEPSI_E_ARG, "null argument");
  *out = nullptr;
  const HostParams& H = sv->P->H;
  const int tbq = std::min<int>(16, std::max<int>(1, (int)sv->max_load));
  // device memory per slot: request + key + sum in NTT form, and tbq pairs of tile buffers
  // (and the request's digit planes when the server holds plaintext planes)
  const size_t per_slot = engine_slot_bytes(H) + tbq * engine_pair_bytes(H) +
                          (sv->plane_groups ? request_plane_bytes(H.consts, H.ell) : 0);
  uint32_t slots = max_active ? max_active : PEPSI_MAX_BATCH;
  if (hbm_budget) slots = (uint32_t)std::min<uint64_t>(slots, hbm_budget / per_slot);
  slots = std::min<uint32_t>(slots, PEPSI_MAX_BATCH);
  if (slots == 0) return fail(PEPSI_E_NOMEM, "HBM budget below one query slot (%zu bytes)", per_slot);
  pepsi_serve* sr = new pepsi_serve();
  sr->sv = sv;
  sr->slots = (int)slots;
  sr->stop_b = std::min<uint32_t>(H.mu, sv->max_load);
  sr->T = (int)((sr->stop_b + tbq - 1) / tbq);
  int rc = sr->eng.setup(sv->P, tbq, (int)slots, sv->need_gen_multi(), sv->values_hat());
  if (!rc && sv->plane_groups) rc = sr->eng.enable_planes(sv->planes_only);
  if (!rc) rc = sr->qslot_dev.ensure(sizeof(int) * slots);
  sr->slot_bytes = per_slot;
  if (!rc && hipHostMalloc((void**)&sr->qslot_host, sizeof(int) * slots * (pepsi_serve::kDepth + 1),
                           hipHostMallocDefault) != hipSuccess)
    rc = fail(PEPSI_E_NOMEM, "pinned slot buffer");
  if (!rc && hipStreamCreateWithFlags(&sr->stream, hipStreamNonBlocking) != hipSuccess)
    rc = fail(PEPSI_E_DEVICE, "stream creation failed");
  if (rc) {
    if (sr->qslot_host) (void)hipHostFree(sr->qslot_host);
    delete sr;
    return rc;
  }
  sr->eng.timer = nullptr;            // the server timer belongs to the calling thread
  sr->active.assign(slots, nullptr);
  sr->worker = std::thread([sr] { sr->loop(); });
  *out = sr;
  return PEPSI_OK;
}

extern "C" int pepsi_serve_submit(pepsi_serve* sr, const uint64_t* cts, const uint64_t* rlk, const uint32_t* mask,
                                  uint64_t* out, uint64_t* req_id) {
  if (!sr || !cts || !rlk || !out || !req_id) return fail(PEPSI_E_ARG, "null argument");
  std::lock_guard<std::mutex> lk(sr->mu);
  if (sr->err) return fail(sr->err, "%s", sr->err_msg.c_str());
  auto* r = new pepsi_serve::Req();
  r->id = sr->next_id++;
  r->cts = cts; r->rlk = rlk; r->mask = mask; r->out = out;
  r->t_submit = now_s();
  sr->reqs[r->id] = r;
  sr->queue.push_back(r);
  *req_id = r->id;
  sr->cv.notify_all();
  return PEPSI_OK;
}

static void fill_stats(const pepsi_serve::Req* r, pepsi_req_stats* st) {
  if (!st) return;
  st->submit_s = r->t_submit;
  st->admit_s = r->t_admit;
  st->done_s = r->t_done;
  st->slot = (uint32_t)r->slot;
  st->done = (uint32_t)r->done;
}

extern "C" int pepsi_serve_poll(pepsi_serve* sr, uint64_t id, int* done, pepsi_req_stats* st) {
  if (!sr || !done) return fail(PEPSI_E_ARG, "null argument");
  std::lock_guard<std::mutex> lk(sr->mu);
  auto it = sr->reqs.find(id);
  if (it == sr->reqs.end()) return fail(PEPSI_E_ARG, "unknown request %llu", (unsigned long long)id);
  *done = it->second->done;
  fill_stats(it->second, st);
  if (sr->err) return fail(sr->err, "%s", sr->err_msg.c_str());
  return PEPSI_OK;
}

extern "C" int pepsi_serve_wait(pepsi_serve* sr, uint64_t id, pepsi_req_stats* st) {
  if (!sr) return fail(PEPSI_E_ARG, "null argument");
  std::unique_lock<std::mutex> lk(sr->mu);
  auto it = sr->reqs.find(id);
  if (it == sr->reqs.end()) return fail(PEPSI_E_ARG, "unknown request %llu", (unsigned long long)id);
  pepsi_serve::Req* r = it->second;
  sr->cv_done.wait(lk, [&] { return r->done || sr->err; });
  fill_stats(r, st);
  if (sr->err) return fail(sr->err, "%s", sr->err_msg.c_str());
  return PEPSI_OK;
}

extern "C" int pepsi_serve_get_info(pepsi_serve* sr, pepsi_serve_info* o) {
  if (!sr || !o) return fail(PEPSI_E_ARG, "null argument");
  std::lock_guard<std::mutex> lk(sr->mu);
  memset(o, 0, sizeof(*o));
  o->slots = (uint32_t)sr->slots;
  o->tiles = (uint32_t)sr->T;
  o->queued = (uint32_t)sr->queue.size();
  for (auto* r : sr->active) o->active += r != nullptr;
  o->steps = sr->steps;
  o->completed = sr->completed;
  o->slot_bytes = sr->slot_bytes;
  return PEPSI_OK;
}

extern "C" void pepsi_serve_destroy(pepsi_serve* sr) {
  if (!sr) return;
  {
    std::lock_guard<std::mutex> lk(sr->mu);
    sr->stop = true;
    sr->cv.notify_all();
  }
  if (sr->worker.joinable()) sr->worker.join();
  if (sr->stream) (void)hipStreamDestroy(sr->stream);
  if (sr->qslot_host) (void)hipHostFree(sr->qslot_host);
  for (hipEvent_t e : sr->ev_pool) (void)hipEventDestroy(e);
  for (auto& st : sr->inflight) (void)hipEventDestroy(st.ev);
  for (auto& kv : sr->reqs) delete kv.second;
  delete sr;
}

// ------------------------------------------------------------------ compression
extern "C" int pepsi_expand_uniform(const pepsi_params* P, const uint8_t* seed, uint32_t first, uint32_t count,
                                    uint64_t* out, uint64_t out_stride, void* stream) {
  if (!P || !seed || (!out && count)) return fail(PEPSI_E_ARG, "null argument");
  const HostParams& H = P->H;
  if (count && out_stride < (uint64_t)H.L * H.n) return fail(PEPSI_E_ARG, "stride below L * N");
  if ((uint64_t)first + count > 0xFFFFFFFFull) return fail(PEPSI_E_ARG, "index range exceeds 32 bits");
  ChaChaKey key;
  for (int i = 0; i < 8; ++i)
    key.k[i] = (uint32_t)seed[4 * i] | (uint32_t)seed[4 * i + 1] << 8 | (uint32_t)seed[4 * i + 2] << 16 |
               (uint32_t)seed[4 * i + 3] << 24;
  expand_uniform(P->T, H.consts, key, (int)first, (int)count, out, (long)out_stride, S(stream));
  HIPCHK(hipGetLastError());
  return PEPSI_OK;
}

extern "C" int pepsi_mod_switch(const pepsi_params* P, const uint64_t* ct, uint64_t* out, void* stream) {
  if (!P || !ct || !out) return fail(PEPSI_E_ARG, "null argument");
  mod_switch(P->T, P->H.consts, ct, out, S(stream));
  HIPCHK(hipGetLastError());
  return PEPSI_OK;
}

// ------------------------------------------------------------------ measurement
extern "C" int pepsi_probe_valu(uint32_t kind, double* lane_ops_per_s) {
  if (!lane_ops_per_s || kind > 6) return fail(PEPSI_E_ARG, "kind must be 0..6 and the output non-null");
  const int rc = probe_valu((int)kind, lane_ops_per_s);
  if (rc == PEPSI_E_NOMEM) return fail(rc, "probe buffer allocation failed");
  if (rc) return fail(rc, "VALU probe failed");
  return PEPSI_OK;
}

// ------------------------------------------------------------------ single steps
extern "C" int pepsi_ntt(const pepsi_params* P, uint64_t* data, uint32_t rows, uint32_t first,
                         uint32_t nprimes, int inverse, void* stream) {
  if (!P || !data) return fail(PEPSI_E_ARG, "null argument");
  const HostParams& H = P->H;
  if (nprimes == 0 || first + nprimes > (uint32_t)(H.L + H.K)) return fail(PEPSI_E_ARG, "bad prime range");
  if (inverse)
    ntt_inverse(P->T, H.logn, data, data, (int)rows, (int)nprimes, (int)first, S(stream));
  else
    ntt_forward(P->T, H.logn, data, LOAD_U64, data, STORE_U64, (int)rows, (int)nprimes, (int)first, S(stream));
  HIPCHK(hipGetLastError());
  return PEPSI_OK;
}

extern "C" int pepsi_encode(const pepsi_params* P, const uint32_t* slots, uint32_t rows, uint32_t* poly,
                            void* stream) {
  if (!P || !slots || !poly) return fail(PEPSI_E_ARG, "null argument");
  encode_slots(P->T, P->H.logn, slots, poly, (int)rows, S(stream));
  HIPCHK(hipGetLastError());
  return PEPSI_OK;
}

extern "C" int pepsi_decode(const pepsi_params* P, const uint32_t* poly, uint32_t rows, uint32_t* slots,
                            void* stream) {
  if (!P || !slots || !poly) return fail(PEPSI_E_ARG, "null argument");
  decode_slots(P->T, P->H.logn, poly, slots, (int)rows, S(stream));
  HIPCHK(hipGetLastError());
  return PEPSI_OK;
}

extern "C" int pepsi_select_sum(const pepsi_params* Pc, const uint64_t* cts, const uint16_t* cw,
                                uint64_t* out, void* stream) {
  pepsi_params* P = const_cast<pepsi_params*>(Pc);
  if (!P || !cts || !cw || !out) return fail(PEPSI_E_ARG, "null argument");
  const HostParams& H = P->H;
  const size_t n = H.n, L = H.L, ell = H.ell;
  // scratch: chat (ell 2 L n) | phat (ell L n) | poly (ell n u32) | S (2 L n)
  const size_t w_c = ell * 2 * L * n, w_p = ell * L * n, w_poly = (ell * n + 1) / 2, w_s = 2 * L * n;
  int rc = P->scratch.ensure((w_c + w_p + w_poly + w_s) * 8);
  if (rc) return rc;
  uint64_t* ch = P->scratch.as<uint64_t>();
  uint64_t* ph = ch + w_c;
  uint32_t* poly = reinterpret_cast<uint32_t*>(ph + w_p);
  uint64_t* Sx = ph + w_p + w_poly;
  hipStream_t s = S(stream);
  ntt_forward(P->T, H.logn, cts, LOAD_U64, ch, STORE_U64, (int)(ell * 2 * L), (int)L, 0, s);
  encode_server_planes(P->T, H.logn, cw, H.h, (int)ell, 0, 1, poly, s);
  PtLayout pl;
  pl.ell = (int)ell;
  pl.gs = 1;
  ntt_forward_plaintexts(P->T, H.logn, poly, ph, 1, (int)L, pl, s);
  select_sum(P->T, H.consts, ch, ph, 1, 0, (int)ell, 1, Sx, (long)(2 * L * n), s);
  ntt_inverse(P->T, H.logn, Sx, out, (int)(2 * L), (int)L, 0, s);
  HIPCHK(hipGetLastError());
  return PEPSI_OK;
}

extern "C" int pepsi_multiply(const pepsi_params* Pc, const uint64_t* x, const uint64_t* y,
                              uint64_t* out, void* stream) {
  pepsi_params* P = const_cast<pepsi_params*>(Pc);
  if (!P || !x || !y || !out) return fail(PEPSI_E_ARG, "null argument");
  const HostParams& H = P->H;
  const size_t n = H.n, L = H.L, K = H.K, Pn = L + K;
  // scratch: xq yq (2 L n each) | xb yb (2 K n each) | d (3 P n)
  const size_t w_q = 2 * L * n, w_b = 2 * K * n, w_d = 3 * Pn * n;
  int rc = P->scratch.ensure((2 * w_q + 2 * w_b + w_d) * 8);
  if (rc) return rc;
  uint64_t* xq = P->scratch.as<uint64_t>();
  uint64_t* yq = xq + w_q;
  uint64_t* xb = yq + w_q;
  uint64_t* yb = xb + w_b;
  uint64_t* dd = yb + w_b;
  hipStream_t s = S(stream);
  ext_q_to_b(P->T, H.consts, x, xb, (long)(K * n), 2, P->fallback.as<uint32_t>(), s);
  ext_q_to_b(P->T, H.consts, y, yb, (long)(K * n), 2, P->fallback.as<uint32_t>(), s);
  ntt_forward(P->T, H.logn, x, LOAD_U64, xq, STORE_U64, (int)(2 * L), (int)L, 0, s);
  ntt_forward(P->T, H.logn, y, LOAD_U64, yq, STORE_U64, (int)(2 * L), (int)L, 0, s);
  ntt_forward(P->T, H.logn, xb, LOAD_U64, xb, STORE_U64, (int)(2 * K), (int)K, (int)L, s);
  ntt_forward(P->T, H.logn, yb, LOAD_U64, yb, STORE_U64, (int)(2 * K), (int)K, (int)L, s);
  TensorJob job{xq, xb, yq, yb, nullptr, nullptr, dd};
  if ((rc = P->job_dev.ensure(sizeof(TensorJob)))) return rc;
  HIPCHK(hipMemcpyAsync(P->job_dev.p, &job, sizeof(job), hipMemcpyHostToDevice, s));
  tensor(P->T, H.consts, P->job_dev.as<TensorJob>(), 1, s);
  ntt_inverse(P->T, H.logn, dd, dd, (int)(3 * Pn), (int)Pn, 0, s);
  scale_round(P->T, H.consts, dd, out, out + 2 * L * n, 1, P->fallback.as<uint32_t>(), s);
  HIPCHK(hipStreamSynchronize(s));       // the job record lives on the host stack
  return PEPSI_OK;
}

extern "C" int pepsi_relin(const pepsi_params* Pc, const uint64_t* ct3, const uint64_t* rlk,
                           uint64_t* out, void* stream) {
  pepsi_params* P = const_cast<pepsi_params*>(Pc);
  if (!P || !ct3 || !rlk || !out) return fail(PEPSI_E_ARG, "null argument");
  const HostParams& H = P->H;
  const size_t n = H.n, L = H.L;
  // scratch: c3h (3 L n) | D (L L n) | rlkh (L 2 L n) | o (2 L n)
  const size_t w_c = 3 * L * n, w_D = L * L * n, w_r = 2 * L * L * n, w_o = 2 * L * n;
  int rc = P->scratch.ensure((w_c + w_D + w_r + w_o) * 8);
  if (rc) return rc;
  uint64_t* c3h = P->scratch.as<uint64_t>();
  uint64_t* Dd = c3h + w_c;
  uint64_t* rh = Dd + w_D;
  uint64_t* o = rh + w_r;
  hipStream_t s = S(stream);
  relin_digits(P->T, H.consts, ct3 + 2 * L * n, Dd, 1, s);
  ntt_forward(P->T, H.logn, Dd, LOAD_U64, Dd, STORE_U64, (int)(L * L), (int)L, 0, s);
  ntt_forward(P->T, H.logn, ct3, LOAD_U64, c3h, STORE_U64, (int)(2 * L), (int)L, 0, s);
  ntt_forward(P->T, H.logn, rlk, LOAD_U64, rh, STORE_U64, (int)(2 * L * L), (int)L, 0, s);
  relin_inner(P->T, H.consts, c3h, Dd, rh, 0, nullptr, 1, 1, 1, o, 1, s);
  ntt_inverse(P->T, H.logn, o, out, (int)(2 * L), (int)L, 0, s);
  HIPCHK(hipGetLastError());
  return PEPSI_OK;
}

// ------------------------------------------------------------------ allocation-free product
// Scratch memory of pepsi_multiply_noalloc: a file-scope device array, of which every GPU the
// library runs on holds its own copy until the process ends.  Its name is a host-side stand-in
// in host code, so host code never passes it to a kernel: it takes each device's address of the
// array from hipGetSymbolAddress on the first call on that device, and uses that address only.
static constexpr size_t kNoAllocScratchBytes = (size_t)8 << 20;
static __device__ __align__(256) uint64_t scratch[kNoAllocScratchBytes / 8];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint64_t* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of the scratch array (looked up once per device).
int scratch_of_current_device(uint64_t** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PEPSI_E_DEVICE, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<uint64_t*>(p);
  }
  *out = g_scratch_ptr[dev];
  return 0;
}
}  // namespace

extern "C" int pepsi_multiply_noalloc(const pepsi_params* P, const uint64_t* x, const uint64_t* y, uint64_t* out,
                                      void* stream) {
  if (!P || !x || !y || !out) return fail(PEPSI_E_ARG, "null argument");
  const HostParams& H = P->H;
  const size_t n = H.n, L = H.L, K = H.K, Pn = L + K;
  const size_t w_q = 2 * L * n, w_b = 2 * K * n, w_d = 3 * Pn * n;
  const size_t need = (2 * w_q + 2 * w_b + w_d) * 8;
  if (need > kNoAllocScratchBytes)
    return fail(PEPSI_E_ARG, "this product needs %zu bytes of scratch; the allocation-free buffer holds %zu "
                "(N = %zu, %zu + %zu primes)", need, kNoAllocScratchBytes, n, L, K);
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev != P->device) return fail(PEPSI_E_ARG, "call on the device the parameters were created on");
  uint64_t* base = nullptr;
  int rc = scratch_of_current_device(&base);
  if (rc) return rc;
  uint64_t* xq = base;
  uint64_t* yq = xq + w_q;
  uint64_t* xb = yq + w_q;
  uint64_t* yb = xb + w_b;
  uint64_t* dd = yb + w_b;
  hipStream_t s = S(stream);
  ext_q_to_b(P->T, H.consts, x, xb, (long)(K * n), 2, P->fallback.as<uint32_t>(), s);
  ext_q_to_b(P->T, H.consts, y, yb, (long)(K * n), 2, P->fallback.as<uint32_t>(), s);
  ntt_forward(P->T, H.logn, x, LOAD_U64, xq, STORE_U64, (int)(2 * L), (int)L, 0, s);
  ntt_forward(P->T, H.logn, y, LOAD_U64, yq, STORE_U64, (int)(2 * L), (int)L, 0, s);
  ntt_forward(P->T, H.logn, xb, LOAD_U64, xb, STORE_U64, (int)(2 * K), (int)K, (int)L, s);
  ntt_forward(P->T, H.logn, yb, LOAD_U64, yb, STORE_U64, (int)(2 * K), (int)K, (int)L, s);
  tensor_one(P->T, H.consts, TensorJob{xq, xb, yq, yb, nullptr, nullptr, dd}, s);
  ntt_inverse(P->T, H.logn, dd, dd, (int)(3 * Pn), (int)Pn, 0, s);
  scale_round(P->T, H.consts, dd, out, out + 2 * L * n, 1, P->fallback.as<uint32_t>(), s);
  HIPCHK(hipGetLastError());
  return PEPSI_OK;
}
