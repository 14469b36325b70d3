"""Pins of the oracle's parameter rules against the paper and number theory."""
import math

import pytest

from oracle import params as P


def test_code_length_paper_value(golden):
    g = golden["code_length_32bit_experiments"]
    assert P.code_length(g["lambda_bar"], g["h"]) == g["ell"]


@pytest.mark.parametrize("lam,h", [(16, 2), (32, 4), (19, 8), (48, 23), (8, 2), (5, 1)])
def test_code_length_is_minimal(lam, h):
    ell = P.code_length(lam, h)
    assert math.comb(ell, h) >= 2 ** lam
    assert math.comb(ell - 1, h) < 2 ** lam


def test_baseline_code_lengths():
    assert P.code_length(32, 4) == 569
    assert P.code_length(16, 2) == 363


def test_comm_optimal_hamming_weight(golden):
    """Sec. 6.1: request size ceil(b/N) * l * N * log2 q is least at h = 8, 8, 23 (b <= 4096)."""
    rows = golden["mod_per_hamming_weight"]["ranges"]

    def table(h):
        for lo, hi, logn, logq in rows:
            if lo <= h <= hi:
                return logn, logq
        raise KeyError(h)

    g = golden["comm_optimal_h"]
    for lam, want in zip(g["lambda_bar"], g["h"]):
        best, best_cost = None, None
        for h in range(1, 65):
            logn, logq = table(h)
            cost = P.code_length(lam, h) * (1 << logn) * logq
            if best_cost is None or cost < best_cost:   # ties keep the smaller h
                best, best_cost = h, cost
        assert best == want


def test_miller_rabin_matches_trial_division():
    def slow(n):
        return n >= 2 and all(n % d for d in range(2, math.isqrt(n) + 1))
    assert all(P.is_prime(n) == slow(n) for n in range(0, 20000))
    for carmichael in (561, 41041, 825265, 321197185, 5394826801, 232250619601, 9746347772161):
        assert not P.is_prime(carmichael)
    assert P.is_prime((1 << 61) - 1) and not P.is_prime((1 << 61) + 1)


@pytest.mark.parametrize("n,count", [(4096, 2), (8192, 4), (16384, 8), (64, 3)])
def test_selected_primes(n, count):
    ps = P.select_primes(n, count)
    assert len(set(ps)) == count and ps == sorted(ps, reverse=True)
    for q in ps:
        assert q < 2 ** 54 and q % (2 * n) == 1 and P.is_prime(q)
    # nothing skipped: every q' = 1 mod 2n between the smallest pick and 2^54 that is prime was picked
    q = ps[-1]
    while q < 2 ** 54:
        if P.is_prime(q):
            assert q in ps
        q += 2 * n
    assert math.prod(ps).bit_length() <= {4096: 109, 8192: 218, 16384: 438, 64: 999}[n]


@pytest.mark.parametrize("n", [16, 4096, 8192, 16384])
def test_primitive_roots(n):
    for q in P.select_primes(n, 2) + [P.T_PLAIN]:
        psi = P.primitive_root_2n(q, n)
        assert pow(psi, n, q) == q - 1          # psi^N = -1
        assert pow(psi, 2 * n, q) == 1          # order exactly 2N (a power of two)


def test_inverse_factorial():
    for h in range(1, 12):
        k = P.inv_factorial_mod_t(h)
        assert k * math.factorial(h) % P.T_PLAIN == 1
    assert P.inv_factorial_mod_t(4) == 19115


def test_server_bin_bound_and_paper_rows(golden):
    assert P.server_mu(256, 4096) == 11
    assert P.server_mu(1 << 22, 8192) == 1870
    for n, b, mu in golden["server_max_bin_load"]["rows"]:
        assert P.server_mu(n, b) == mu
        # the paper's loads sit above the mean load 3n/b and at or below the 2^-40 union bound
        assert 3 * n / b < mu <= P.server_bin_bound(n, b)


@pytest.mark.parametrize("n_items,n_bins", [(0, 1024), (1, 1024), (2, 64), (5, 16), (9, 8)])
def test_server_bin_bound_small_sets_exact(n_items, n_bins):
    """Tiny sets, where the load can reach every trial: the bound equals the least mu whose
    exact binomial tail (rational arithmetic over all 3 n outcomes) passes the 2^-40 test."""
    from fractions import Fraction
    trials, p = 3 * n_items, Fraction(1, n_bins)
    pmf = [math.comb(trials, j) * p ** j * (1 - p) ** (trials - j) for j in range(trials + 1)]
    mu = 0
    while n_bins * sum(pmf[mu:]) > Fraction(1, 2 ** 40):
        mu += 1
    assert P.server_bin_bound(n_items, n_bins) == mu
    assert mu >= (1 if n_items == 0 else 2)
