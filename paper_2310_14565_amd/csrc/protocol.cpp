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

void place(uint32_t x, int i, uint64_t seed, uint32_t nbins, int pbh_bits, uint32_t* bin, uint32_t* value) {
  if (!pbh_bits) {
    *bin = hash_bin(x, i, seed, nbins);
    *value = x;
    return;
  }
  int c = 0;
  while ((1u << c) < nbins) ++c;
  const int low = pbh_bits - c;
  const uint32_t xl = low >= 32 ? x : (x & ((1u << low) - 1));
  const uint32_t xh = low >= 32 ? 0 : (x >> low);
  *bin = xh ^ hash_bin(xl, i, seed, nbins);
  *value = ((uint32_t)(i - 1) << low) | xl;
}

int cuckoo_insert(const uint32_t* items, uint64_t m, uint32_t nbins, uint64_t seed, int k,
                  int max_evictions, uint32_t* table, uint8_t* valid, int pbh_bits) {
  std::vector<uint8_t> which(nbins, 0);   // hash function (1..k) an occupant sits under; 0 = empty
  for (uint32_t b = 0; b < nbins; ++b) { table[b] = 0; valid[b] = 0; }
  for (uint64_t n = 0; n < m; ++n) {
    uint32_t cur = items[n];
    int idx = 1, evictions = 0;
    for (;;) {
      uint32_t pos, val;
      place(cur, idx, seed, nbins, pbh_bits, &pos, &val);
      if (!which[pos]) {
        table[pos] = cur;
        which[pos] = (uint8_t)idx;
        valid[pos] = 1;
        break;
      }
      const uint32_t ev = table[pos];
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

int simple_hash(const uint32_t* items, uint64_t n, uint32_t nbins, uint64_t seed, int k, uint32_t mu,
                std::vector<uint32_t>* table, std::vector<uint8_t>* valid, uint32_t* max_load,
                std::vector<uint32_t>* index, int pbh_bits) {
  std::vector<uint32_t> load(nbins, 0);
  table->assign((size_t)mu * nbins, 0);
  valid->assign((size_t)mu * nbins, 0);
  if (index) index->assign((size_t)mu * nbins, 0);
  uint32_t bins[8], vals[8];
  for (uint64_t e = 0; e < n; ++e) {
    const uint32_t y = items[e];
    int nb = 0;
    for (int i = 1; i <= k; ++i) {
      uint32_t b, v;
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
