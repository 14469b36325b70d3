"""Host-side checks of the word arithmetic the GPU kernels are built on (csrc/modarith.hpp).

The header's functions are host- and device-callable; here they are compiled for the host with g++
(a two-line stand-in replaces the HIP runtime header) and checked against 128-bit arithmetic on
random and extreme inputs, for primes of the kind the library uses (p = 1 mod 2^15, 2^53 < p < 2^54):
- shoup_lazy4, the NTT butterfly product with a quotient from three partial products: congruent to
  x w mod p and below 4p for every 64-bit x;
- shoup_lazy: congruent and below 2p; shoup: fully reduced;
- reduce116: exact for every value below 2^116; reduce116_lazy: congruent and below 3p.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2310_14565_amd", "csrc")

PROGRAM = r"""
#include "modarith.hpp"
#include <cstdio>
#include <random>
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
int main() {
  std::mt19937_64 g(2310);
  const uint64_t step = 1ull << 15;
  uint64_t ps[4]; int np = 0;
  for (uint64_t q = ((1ull << 54) - 1) / step * step + 1; np < 3; q -= step) if (is_prime(q)) ps[np++] = q;
  for (uint64_t q = (1ull << 53) / step * step + 1 + step; np < 4; q += step) if (is_prime(q)) ps[np++] = q;
  long bad = 0, n = 0;
  for (int pi = 0; pi < 4; ++pi) {
    const uint64_t p = ps[pi];
    Prime P; P.p = p; P.barrett = (uint64_t)(((u128)1 << 116) / p); P.r64 = (uint64_t)(((u128)1 << 64) % p);
    for (int it = 0; it < 400000; ++it) {
      uint64_t w = g() % p;
      if (it % 11 == 0) w = (it / 11) % 3 == 0 ? 0 : (it / 11) % 3 == 1 ? 1 : p - 1;
      uint64_t x;
      switch (it % 5) {
        case 0: x = g(); break;
        case 1: x = g() % (57 * p); break;
        case 2: x = ~0ull - g() % 4096; break;
        case 3: x = (g() % 64) * p + g() % 3 - (it & 1); break;
        default: x = g() >> (g() % 64); break;
      }
      const uint64_t wq = shoup_companion(w, p);
      const uint64_t want = (uint64_t)((u128)x * w % p);
      const uint64_t r4 = shoup_lazy4(x, w, wq, p), r2 = shoup_lazy(x, w, wq, p), r1 = shoup(x, w, wq, p);
      ++n;
      if (r4 >= 4 * p || r4 % p != want) ++bad;
      if (r2 >= 2 * p || r2 % p != want) ++bad;
      if (r1 != want) ++bad;
      const u128 v = ((u128)(g() >> 12) << 64 | g()) >> (g() % 40);   // below 2^116
      if (reduce116((uint64_t)v, (uint64_t)(v >> 64), P) != (uint64_t)(v % p)) ++bad;
      const uint64_t rl = reduce116_lazy((uint64_t)v, (uint64_t)(v >> 64), P);
      if (rl >= 3 * p || rl % p != (uint64_t)(v % p)) ++bad;
    }
  }
  printf("checked %ld bad %ld\n", n, bad);
  return bad != 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_modarith_host():
    with tempfile.TemporaryDirectory() as d:
        os.makedirs(os.path.join(d, "hip"))
        with open(os.path.join(d, "hip", "hip_runtime.h"), "w") as f:
            f.write("#pragma once\n#define __host__\n#define __device__\n#define __forceinline__ inline\n")
        src = os.path.join(d, "t.cpp")
        with open(src, "w") as f:
            f.write(PROGRAM)
        exe = os.path.join(d, "t")
        subprocess.run(["g++", "-O2", "-std=c++17", "-I", d, "-I", CSRC, src, "-o", exe], check=True,
                       capture_output=True, text=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "bad 0" in r.stdout
