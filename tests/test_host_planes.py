"""Host-side checks of the exact int8 digit-plane contraction (csrc/planes.hpp) that the batched
select-and-sum runs on the matrix cores.

The header is compiled for the host with g++ (a stand-in replaces the HIP runtime header), the
matrix products are replaced by a plain loop over the digit products with 64-bit sums, and every
quantity the exactness argument bounds is checked against its bound at the largest admitted code
length, with extreme and random residues, for primes of the kind the library uses:
- the seven balanced base-256 digits give back the residue, with |d_i| <= 128 and the top digit in
  [0, 64];
- every weight sum |T_s| < 2^31 (an int32 accumulator is exact) and every group |V_g| < 2^53;
- the recombined residue equals sum_j x_j y_j mod p computed with 128-bit integers;
- planes_supported admits exactly the code lengths 1 .. 4096.
Dropping a digit or a weight of the recombination makes the residue check fail.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2310_14565_amd", "csrc")

PROGRAM = r"""
#include "planes.hpp"
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>
using namespace pepsi;
static bool is_prime(uint64_t n) {
  if (n < 2) return false;
  for (uint64_t q : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull})
    if (n % q == 0) return n == q;
  uint64_t d = n - 1; int s = 0;
  while (!(d & 1)) { d >>= 1; ++s; }
  auto pw = [&](uint64_t a, uint64_t e) { u128 r = 1, b = a; while (e) { if (e & 1) r = r * b % n; b = b * b % n; e >>= 1; } return (uint64_t)r; };
  for (uint64_t a : {2ull, 3ull, 5ull, 7ull, 11ull, 13ull, 17ull, 19ull, 23ull, 29ull, 31ull, 37ull}) {
    uint64_t x = pw(a, d);
    if (x == 1 || x == n - 1) continue;
    bool ok = false;
    for (int r = 1; r < s; ++r) { x = (uint64_t)((u128)x * x % n); if (x == n - 1) { ok = true; break; } }
    if (!ok) return false;
  }
  return true;
}
// the value whose six low balanced digits all equal d and whose top digit is top
static uint64_t with_digits(int d, int top) {
  int64_t v = (int64_t)top << 48;
  for (int i = 0; i < 6; ++i) v += (int64_t)d << (8 * i);
  return (uint64_t)v;
}
int main(int argc, char** argv) {
  const int drop = argc > 1 ? atoi(argv[1]) : -1;   // planted mistake: skip one weight
  std::mt19937_64 g(2310);
  const uint64_t step = 1ull << 15;
  uint64_t ps[3]; int np = 0;
  for (uint64_t q = ((1ull << 54) - 1) / step * step + 1; np < 2; q -= step) if (is_prime(q)) ps[np++] = q;
  for (uint64_t q = (1ull << 53) / step * step + 1 + step; np < 3; q += step) if (is_prime(q)) ps[np++] = q;
  long bad = 0, checks = 0;
  int64_t maxT = 0, maxV = 0;
  // digits
  for (int it = 0; it < 2000000; ++it) {
    uint64_t x = it < 8 ? (uint64_t[]){0, 1, 127, 128, 255, (1ull << 54) - 1, (1ull << 53), ps[0] - 1}[it]
                        : g() >> 10;
    int8_t d[PL_DG];
    balanced_digits(x, d);
    int64_t back = 0;
    for (int i = PL_DG - 1; i >= 0; --i) back = back * 256 + d[i];
    ++checks;
    if ((uint64_t)back != x || d[PL_DG - 1] < 0 || d[PL_DG - 1] > 64) ++bad;
  }
  const int ell = PL_MAX_ELL;
  std::vector<uint64_t> x(ell), y(ell);
  for (int pi = 0; pi < np; ++pi) {
    const uint64_t p = ps[pi];
    Prime P; P.p = p; P.barrett = (uint64_t)(((u128)1 << 116) / p); P.r64 = (uint64_t)(((u128)1 << 64) % p);
    uint64_t wgt[4];
    plane_group_weights(P, wgt);
    for (int trial = 0; trial < 12; ++trial) {
      for (int j = 0; j < ell; ++j) {
        switch (trial) {
          case 0: x[j] = y[j] = with_digits(-128, 32); break;          // every digit product +2^14
          case 1: x[j] = with_digits(-128, 32); y[j] = with_digits(127, 31); break;   // -127 * 128
          case 2: x[j] = y[j] = p - 1; break;
          case 3: x[j] = p - 1; y[j] = 0; break;
          case 4: x[j] = y[j] = (j & 1) ? with_digits(-128, 32) : with_digits(127, 31); break;
          default: x[j] = g() % p; y[j] = (trial % 3 == 0) ? p - 1 - (g() % 1024) : g() % p; break;
        }
        if (x[j] >= p || y[j] >= p) { printf("bad test value\n"); return 2; }
      }
      int64_t T[PL_WEIGHTS] = {0};
      u128 want = 0;
      for (int j = 0; j < ell; ++j) {
        int8_t a[PL_DG], b[PL_DG];
        balanced_digits(x[j], a);
        balanced_digits(y[j], b);
        for (int u = 0; u < PL_DG; ++u)
          for (int v = 0; v < PL_DG; ++v) T[u + v] += (int64_t)a[u] * b[v];
        want += (u128)x[j] * y[j];
      }
      int32_t T32[PL_WEIGHTS];
      for (int s = 0; s < PL_WEIGHTS; ++s) {
        if (llabs(T[s]) > maxT) maxT = llabs(T[s]);
        if (llabs(T[s]) >= (1ll << 31)) ++bad;
        T32[s] = s == drop ? 0 : (int32_t)T[s];
      }
      for (int gi = 0; gi < 4; ++gi) {
        int64_t V = 0;
        for (int s = 4 * gi; s < 4 * gi + 4 && s < PL_WEIGHTS; ++s) V += T[s] << (8 * (s - 4 * gi));
        if (llabs(V) > maxV) maxV = llabs(V);
        if (llabs(V) >= (1ll << 53)) ++bad;
      }
      ++checks;
      if (plane_recombine(T32, P, wgt) != (uint64_t)(want % p)) ++bad;
    }
  }
  for (int e : {0, 1, 4096, 4097, 65534}) {
    ++checks;
    if (planes_supported(e) != (e >= 1 && e <= 4096)) ++bad;
  }
  printf("checked %ld bad %ld max|T| 2^%.3f max|V| 2^%.3f\n", checks, bad, __builtin_log2((double)maxT),
         __builtin_log2((double)maxV));
  return bad != 0;
}
"""


def _build(d):
    os.makedirs(os.path.join(d, "hip"))
    with open(os.path.join(d, "hip", "hip_runtime.h"), "w") as f:
        f.write("#pragma once\n#define __host__\n#define __device__\n#define __forceinline__ inline\n")
    src = os.path.join(d, "t.cpp")
    with open(src, "w") as f:
        f.write(PROGRAM)
    exe = os.path.join(d, "t")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", d, "-I", CSRC, src, "-o", exe], check=True,
                   capture_output=True, text=True)
    return exe


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_digit_planes_exact_at_max_code_length():
    with tempfile.TemporaryDirectory() as d:
        exe = _build(d)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "bad 0" in r.stdout
        # the extreme cases reach the bounds' order: |T_s| within 2^31 and |V_g| within 2^53
        line = r.stdout.split()
        assert float(line[line.index("max|T|") + 1][2:]) > 28.5
        assert float(line[line.index("max|V|") + 1][2:]) > 52.0
        # a planted mistake (one weight sum dropped) is caught
        for drop in (0, 6, 12):
            r = subprocess.run([exe, str(drop)], capture_output=True, text=True, timeout=300)
            assert r.returncode != 0 and "bad 0" not in r.stdout
