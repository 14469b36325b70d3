// Host-side protocol preparation: hashing to bins and constant-weight codes.
#pragma once
#include <stdint.h>
#include <vector>
#include "modarith.hpp"

namespace pepsi {

uint64_t mix64(uint64_t z);                       // SplitMix64 output finaliser
// H_i(x) = mix64(x ^ (seed + i * 0x9E3779B97F4A7C15)) mod nbins, i = 1..k
uint32_t hash_bin(uint64_t x, int i, uint64_t seed, uint32_t nbins);

// Bin and stored value of x under hash function i.  pbh_bits = 0: (H_i(x), x).  Permutation-
// based hashing (Sec. 3.3) with pbh_bits = lambda and nbins = 2^c, x = x_H || x_L, |x_L| =
// lambda - c: (x_H ^ H_i(x_L), (i - 1) 2^(lambda - c) + x_L) -- the stored value names the hash
// function, so equal values in equal bins mean equal elements with k > 1 hash functions.
// Elements and values are up to 64 bits (32-bit elements, or large elements hashed to lambda
// bits).
void place(uint64_t x, int i, uint64_t seed, uint32_t nbins, int pbh_bits, uint32_t* bin, uint64_t* value);

// Cuckoo hashing without a stash; table receives each bin's stored value; returns 0 or -3
// (eviction limit exceeded).
int cuckoo_insert(const uint64_t* items, uint64_t m, uint32_t nbins, uint64_t seed, int k,
                  int max_evictions, uint64_t* table, uint8_t* valid, int pbh_bits = 0);
// Every element to each distinct bin among H_1..H_k (with PBH: one entry per hash function,
// since the k stored values differ), input order; table/valid [mu][nbins]; with index non-null
// also the element's input position per entry; returns 0 or -4 (a bin exceeds mu).
int simple_hash(const uint64_t* items, uint64_t n, uint32_t nbins, uint64_t seed, int k, uint32_t mu,
                std::vector<uint64_t>* table, std::vector<uint8_t>* valid, uint32_t* max_load,
                std::vector<uint32_t>* index = nullptr, int pbh_bits = 0);

// Large elements (Sec. 5, "Optimization for Large Elements"): the first `bits` bits (1..64) of
// SHA-256 (FIPS 180-4) of a byte string, read big-endian.
uint64_t hash_element(const uint8_t* data, uint64_t len, int bits);

// Constant-weight code CW(ell, h) by the combinatorial number system.
class CwEncoder {
 public:
  CwEncoder(int ell, int h);
  void encode(uint64_t v, uint16_t* pos) const;   // h positions, descending
 private:
  int ell_, h_;
  std::vector<uint64_t> binom_;
};

}  // namespace pepsi
