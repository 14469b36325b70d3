// Exact int8 digit planes of 54-bit residues, for the select-and-sum of many queries on the
// int8 matrix cores.  Host- and device-callable, so that the exactness argument below can be
// checked on the host.
//
// A residue x < 2^54 is written as seven balanced base-256 digits x = sum_i d_i 256^i with
// d_i in [-128, 127] for i < 6 and the top digit d_6 in [0, 64].  For one output, the products
// of a client and a server residue summed over the ell code positions are
//   sum_j x_j y_j = sum_{s=0}^{12} T_s 256^s,  T_s = sum_j sum_{u+v=s} d_u(x_j) d_v(y_j),
// and each T_s has at most 7 digit products per position, each of magnitude at most 2^14
// (128 * 128), so |T_s| <= 7 ell 2^14 < 2^31 for ell <= PL_MAX_ELL: the int32 accumulators of
// the matrix instructions are exact.  The 13 weight sums are recombined in four groups of four
// weights, V_g = sum_{s=4g}^{4g+3} T_s 256^(s - 4g), with |V_g| <= 7 ell 2^14 (1 + 2^8 + 2^16 +
// 2^24) < 2^53 <= p for ell <= PL_MAX_ELL, so V_g + p lies in [0, 2p) and
//   sum_j x_j y_j = sum_g V_g 2^(32 g)   (mod p)
// is a sum of four products, each below 2p * p < 2^109, so below 2^111: one 116-bit Barrett
// reduction.
#pragma once
#include "modarith.hpp"

namespace pepsi {

constexpr int PL_DG = 7, PL_K = 64, PL_MAX_ELL = 4096;
constexpr int PL_WEIGHTS = 2 * PL_DG - 1;

// Whether a code length keeps every weight sum and group exact (the bounds above).
PEPSI_HD bool planes_supported(int ell) { return ell > 0 && ell <= PL_MAX_ELL; }

PEPSI_HD void balanced_digits(uint64_t x, int8_t (&d)[PL_DG]) {
#pragma unroll
  for (int i = 0; i < PL_DG - 1; ++i) {
    int v = (int)(x & 255);
    v -= v >= 128 ? 256 : 0;
    d[i] = (int8_t)v;
    x = (x - (uint64_t)(int64_t)v) >> 8;
  }
  d[PL_DG - 1] = (int8_t)x;     // at most 64 for x < 2^54
}

// The four factors 2^(32 g) mod p, g = 0..3.
PEPSI_HD void plane_group_weights(const Prime& pr, uint64_t (&wgt)[4]) {
  wgt[0] = 1;
  wgt[1] = 1ull << 32;
  wgt[2] = pr.r64;
  wgt[3] = mulmod(pr.r64, 1ull << 32, pr);
}

// sum_s T_s 256^s mod p from the 13 exact weight sums.
PEPSI_HD uint64_t plane_recombine(const int32_t (&T)[PL_WEIGHTS], const Prime& pr, const uint64_t (&wgt)[4]) {
  u128 tot = 0;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    int64_t V = 0;
#pragma unroll
    for (int s = 4 * g; s < 4 * g + 4 && s < PL_WEIGHTS; ++s) V += (int64_t)T[s] << (8 * (s - 4 * g));
    tot += (u128)(uint64_t)(V + (int64_t)pr.p) * wgt[g];
  }
  return reduce116((uint64_t)tot, (uint64_t)(tot >> 64), pr);   // tot < 4 (2p) p < 2^111
}

}  // namespace pepsi
