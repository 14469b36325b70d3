// Host-side protocol preparation: hashing to bins and constant-weight codes.
#pragma once
#include <stdint.h>
#include <vector>
#include "modarith.hpp"

namespace pepsi {

uint64_t mix64(uint64_t z);                       // SplitMix64 output finaliser
// H_i(x) = mix64(x ^ (seed + i * 0x9E3779B97F4A7C15)) mod nbins, i = 1..k
uint32_t hash_bin(uint64_t x, int i, uint64_t seed, uint32_t nbins);

// Cuckoo hashing without a stash; returns 0 or -3 (eviction limit exceeded).
int cuckoo_insert(const uint32_t* items, uint64_t m, uint32_t nbins, uint64_t seed, int k,
                  int max_evictions, uint32_t* table, uint8_t* valid);
// Every element to each distinct bin among H_1..H_k, input order; table/valid [mu][nbins];
// with index non-null also the element's input position per entry; returns 0 or -4 (a bin
// exceeds mu).
int simple_hash(const uint32_t* items, uint64_t n, uint32_t nbins, uint64_t seed, int k, uint32_t mu,
                std::vector<uint32_t>* table, std::vector<uint8_t>* valid, uint32_t* max_load,
                std::vector<uint32_t>* index = nullptr);

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
