// Host-side protocol preparation (Sec. 3.2, 3.3, 4.1; Alg. 6): hashing to
// bins and constant-weight encoding.  Plain sequential C++; the GPU only sees
// the resulting codeword positions.
#include "protocol.hpp"

#include <algorithm>
#include <vector>

namespace pepsi {

uint64_t mix64(uint64_t z) {
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return z;
}

uint32_t hash_bin(uint64_t x, int i, uint64_t seed, uint32_t nbins) {
  return (uint32_t)(mix64(x ^ (seed + (uint64_t)i * 0x9E3779B97F4A7C15ull)) % nbins);
}

void place(uint64_t x, int i, uint64_t seed, uint32_t nbins, int pbh_bits, uint32_t* bin, uint64_t* value) {
  if (!pbh_bits) {
    *bin = hash_bin(x, i, seed, nbins);
    *value = x;
    return;
  }
  int c = 0;
  while ((1u << c) < nbins) ++c;
  const int low = pbh_bits - c;
  const uint64_t xl = low >= 64 ? x : (x & ((1ull << low) - 1));
  const uint64_t xh = low >= 64 ? 0 : (x >> low);
  *bin = (uint32_t)xh ^ hash_bin(xl, i, seed, nbins);
  *value = ((uint64_t)(i - 1) << low) | xl;
}

int cuckoo_insert(const uint64_t* items, uint64_t m, uint32_t nbins, uint64_t seed, int k,
                  int max_evictions, uint64_t* table, uint8_t* valid, int pbh_bits) {
  std::vector<uint8_t> which(nbins, 0);   // hash function (1..k) an occupant sits under; 0 = empty
  for (uint32_t b = 0; b < nbins; ++b) { table[b] = 0; valid[b] = 0; }
  for (uint64_t n = 0; n < m; ++n) {
    uint64_t cur = items[n];
    int idx = 1, evictions = 0;
    for (;;) {
      uint32_t pos;
      uint64_t val;
      place(cur, idx, seed, nbins, pbh_bits, &pos, &val);
      if (!which[pos]) {
        table[pos] = cur;
        which[pos] = (uint8_t)idx;
        valid[pos] = 1;
        break;
      }
      const uint64_t ev = table[pos];
      const int ev_idx = which[pos];
      table[pos] = cur;
      which[pos] = (uint8_t)idx;
      cur = ev;
      idx = ev_idx % k + 1;
      if (++evictions > max_evictions) return -3;
    }
  }
  if (pbh_bits)                            // the table keeps the elements until here
    for (uint32_t b = 0; b < nbins; ++b)
      if (which[b]) {
        uint32_t pos;
        place(table[b], which[b], seed, nbins, pbh_bits, &pos, &table[b]);
      }
  return 0;
}

int simple_hash(const uint64_t* items, uint64_t n, uint32_t nbins, uint64_t seed, int k, uint32_t mu,
                std::vector<uint64_t>* table, std::vector<uint8_t>* valid, uint32_t* max_load,
                std::vector<uint32_t>* index, int pbh_bits) {
  std::vector<uint32_t> load(nbins, 0);
  table->assign((size_t)mu * nbins, 0);
  valid->assign((size_t)mu * nbins, 0);
  if (index) index->assign((size_t)mu * nbins, 0);
  uint32_t bins[8];
  uint64_t vals[8];
  for (uint64_t e = 0; e < n; ++e) {
    const uint64_t y = items[e];
    int nb = 0;
    for (int i = 1; i <= k; ++i) {
      uint32_t b;
      uint64_t v;
      place(y, i, seed, nbins, pbh_bits, &b, &v);
      bool dup = false;
      if (!pbh_bits)
        for (int q = 0; q < nb; ++q) dup |= bins[q] == b;
      if (!dup) { bins[nb] = b; vals[nb] = v; ++nb; }
    }
    for (int q = 0; q < nb; ++q) {
      const uint32_t b = bins[q];
      if (load[b] >= mu) return -4;
      (*table)[(size_t)load[b] * nbins + b] = vals[q];
      (*valid)[(size_t)load[b] * nbins + b] = 1;
      if (index) (*index)[(size_t)load[b] * nbins + b] = (uint32_t)e;
      ++load[b];
    }
  }
  *max_load = 0;
  for (uint32_t b = 0; b < nbins; ++b) *max_load = std::max(*max_load, load[b]);
  return 0;
}

// ---- SHA-256 (FIPS 180-4) ----
namespace {
// The constants are derived from their definition: the first 32 bits of the fractional parts of
// the cube roots (K) and square roots (initial hash value) of the first 64 (8) primes, i.e.
// floor(root(p) 2^32) mod 2^32, computed with integer roots.
uint64_t iroot(u128 v, int k) {                    // floor(v^(1/k)) for k = 2, 3 and v < 2^106
  uint64_t lo = 0, hi = (uint64_t)1 << 36;         // the roots here are below 2^36, so hi^k < 2^128
  while (lo < hi) {
    const uint64_t mid = lo + (hi - lo + 1) / 2;
    u128 p = 1;
    for (int r = 0; r < k; ++r) p *= mid;
    if (p <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}
struct ShaConsts {
  uint32_t K[64], H0[8];
  ShaConsts() {
    int found = 0;
    for (uint32_t p = 2; found < 64; ++p) {
      bool prime = true;
      for (uint32_t d = 2; d * d <= p; ++d) prime &= p % d != 0;
      if (!prime) continue;
      K[found] = (uint32_t)iroot((u128)p << 96, 3);
      if (found < 8) H0[found] = (uint32_t)iroot((u128)p << 64, 2);
      ++found;
    }
  }
};
const ShaConsts& sha_consts() {
  static const ShaConsts c;
  return c;
}
inline uint32_t rotr(uint32_t x, int r) { return (x >> r) | (x << (32 - r)); }
void sha_block(uint32_t (&h)[8], const uint8_t* blk, const ShaConsts& C) {
  uint32_t w[64];
  for (int t = 0; t < 16; ++t)
    w[t] = (uint32_t)blk[4 * t] << 24 | (uint32_t)blk[4 * t + 1] << 16 | (uint32_t)blk[4 * t + 2] << 8 | blk[4 * t + 3];
  for (int t = 16; t < 64; ++t) {
    const uint32_t s0 = rotr(w[t - 15], 7) ^ rotr(w[t - 15], 18) ^ (w[t - 15] >> 3);
    const uint32_t s1 = rotr(w[t - 2], 17) ^ rotr(w[t - 2], 19) ^ (w[t - 2] >> 10);
    w[t] = w[t - 16] + s0 + w[t - 7] + s1;
  }
  uint32_t a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], hh = h[7];
  for (int t = 0; t < 64; ++t) {
    const uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
    const uint32_t ch = (e & f) ^ (~e & g);
    const uint32_t t1 = hh + S1 + ch + C.K[t] + w[t];
    const uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
    const uint32_t maj = (a & b) ^ (a & c) ^ (b & c);
    const uint32_t t2 = S0 + maj;
    hh = g; g = f; f = e; e = d + t1; d = c; c = b; b = a; a = t1 + t2;
  }
  h[0] += a; h[1] += b; h[2] += c; h[3] += d; h[4] += e; h[5] += f; h[6] += g; h[7] += hh;
}
}  // namespace

uint64_t hash_element(const uint8_t* data, uint64_t len, int bits) {
  const ShaConsts& C = sha_consts();
  uint32_t h[8];
  for (int i = 0; i < 8; ++i) h[i] = C.H0[i];
  uint64_t off = 0;
  for (; off + 64 <= len; off += 64) sha_block(h, data + off, C);
  // padding: 0x80, zeros, and the bit length as a 64-bit big-endian integer
  uint8_t tail[128] = {0};
  const uint64_t rem = len - off;
  for (uint64_t i = 0; i < rem; ++i) tail[i] = data[off + i];
  tail[rem] = 0x80;
  const int blocks = rem + 9 <= 64 ? 1 : 2;
  const uint64_t bitlen = len * 8;
  for (int i = 0; i < 8; ++i) tail[64 * blocks - 1 - i] = (uint8_t)(bitlen >> (8 * i));
  for (int b = 0; b < blocks; ++b) sha_block(h, tail + 64 * b, C);
  const uint64_t top = (uint64_t)h[0] << 32 | h[1];
  return bits >= 64 ? top : top >> (64 - bits);
}

CwEncoder::CwEncoder(int ell, int h) : ell_(ell), h_(h), binom_((size_t)(h + 1) * ell, 0) {
  // binom_[r][c] = C(c, r), saturated at 2^64 - 1 (only values <= the encoded value matter)
  for (int r = 0; r <= h; ++r)
    for (int c = 0; c < ell; ++c) {
      u128 v = 1;
      bool sat = false;
      if (c < r) v = 0;
      for (int q = 0; q < r && c >= r; ++q) {
        v = v * (u128)(c - q) / (u128)(q + 1);
        if (v >> 64) { sat = true; break; }
      }
      binom_[(size_t)r * ell + c] = sat ? ~0ull : (uint64_t)v;
    }
}

// Positions c_h > ... > c_1 with v = sum_r C(c_r, r): c_r is the largest c with C(c, r) <= v.
void CwEncoder::encode(uint64_t v, uint16_t* pos) const {
  for (int r = h_, out = 0; r >= 1; --r, ++out) {
    const uint64_t* row = &binom_[(size_t)r * ell_];
    int lo = r - 1, hi = ell_ - 1;          // C(r-1, r) = 0 <= v always
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (row[mid] <= v) lo = mid; else hi = mid - 1;
    }
    pos[out] = (uint16_t)lo;
    v -= row[lo];
  }
}

}  // namespace pepsi
