"""Oracle (test infrastructure only): large elements (Sec. 5, "Optimization for Large Elements",
Lemma "fail-collide"; Sec. 7, "Parameters for Large Elements").

Elements of any length (byte strings) are not compared homomorphically.  Each is first mapped to
a lambda-bit value with a hash function, and the protocol runs on those values.  Two unequal
elements then match only if their values collide and they are compared, i.e. a client and a
server element sit in one bin.  A bin holds at most mu_c client and mu_s server entries, so over
b bins at most b mu_c mu_s pairs are compared, each colliding with probability 2^-lambda for a
random hash function (the Lemma):

    P[failure] <= b mu_c mu_s / 2^lambda,

and the paper takes lambda = alpha + ceil(log2(b mu_c mu_s)) for a failure rate of at most
2^-alpha, with alpha = 40 and mu_c = 1 (cuckoo hashing without a stash).

Readings (the paper does not fix them):
* The hash function: the first lambda bits of SHA-256 (FIPS 180-4) of the element, read as a
  big-endian integer (lambda <= 64 here).
* The code: the paper uses a lossy constant-weight mapping for large elements, from its
  reference, without giving the algorithm.  Here the values go through permutation-based hashing
  as for 32-bit elements (with the hash-function index in the stored value) and the perfect
  mapping (the combinatorial number system) over the stored bits.  The lossy mapping would trade
  a shorter code for further false matches; the perfect one adds none, so the Lemma's bound is
  the failure rate of the whole protocol.
* The Hamming weight: not stated for large elements.  With b = N = 16384 (Sec. 7), Table
  "mod-per-hamming-weight" places h in 9..32; h = 16 is the weight the paper's own discussion
  of effective bitlength 48 names as much cheaper to compute than the communication optimum 23
  for under 6% more communication (Sec. 6).
"""
from __future__ import annotations

import hashlib
import math
import random
from fractions import Fraction

import numpy as np

from . import hashing

ALPHA = 40          # Sec. 7: failure rate below 2^-40


def ceil_log2(x: int) -> int:
    """ceil(log2 x) for an integer x >= 1, exactly."""
    assert x >= 1
    return (x - 1).bit_length()


def element_bits(n_bins: int, mu_client: int, mu_server: int, alpha: int = ALPHA) -> int:
    """lambda = alpha + ceil(log2(b mu_c mu_s)) (Sec. 5, after the Lemma)."""
    return alpha + ceil_log2(n_bins * mu_client * mu_server)


def failure_bound(n_bins: int, mu_client: int, mu_server: int, lam: int) -> Fraction:
    """The Lemma's bound b mu_c mu_s / 2^lambda, exactly."""
    return Fraction(n_bins * mu_client * mu_server, 1 << lam)


def hash_to_bits(element: bytes, lam: int) -> int:
    """The first lam bits of SHA-256(element), big-endian (1 <= lam <= 64)."""
    assert 1 <= lam <= 64
    return int.from_bytes(hashlib.sha256(element).digest()[:8], "big") >> (64 - lam)


def hash_elements(elements, lam: int) -> np.ndarray:
    return np.array([hash_to_bits(e, lam) for e in elements], dtype=np.uint64)


def random_elements(count: int, length: int, seed: int, exclude=()) -> list[bytes]:
    """count distinct random byte strings of the given length (none of them in exclude)."""
    g = random.Random(seed)
    seen = set(exclude)
    out = []
    while len(out) < count:
        e = bytes(g.getrandbits(8) for _ in range(length))
        if e not in seen:
            seen.add(e)
            out.append(e)
    return out


def table_matches(client_values, server_values, n_bins: int, lam: int, mu: int, seed: int = 0x5EED,
                  n_hash: int = 3) -> int:
    """The protocol's hashing on lam-bit values (cuckoo table of the client's distinct values,
    simple table of the server's, permutation-based hashing over lam bits): the number of bins
    in which the client's entry equals one of the server's entries, i.e. the matches the
    encrypted comparison finds."""
    cvals = list(dict.fromkeys(int(v) for v in client_values))   # a client-side collision is one item
    table, valid = hashing.cuckoo_table(cvals, n_bins, seed, n_hash, pbh_bits=lam)
    stab, svalid, _ = hashing.simple_table(np.array([int(v) for v in server_values], dtype=np.uint64), n_bins,
                                           mu, seed, n_hash, pbh_bits=lam)
    hit = (stab == table[None, :]) & svalid.astype(bool) & valid.astype(bool)[None, :]
    return int(hit.any(axis=0).sum())
