"""Oracle (test infrastructure only): parameters of the scheme and the protocol.

Every rule here is written from its definition with Python integers:

* ``code_length``: eq. (1) of Sec. 4.1, the least l with C(l, h) >= 2^lambda_bar.
* ``select_primes``: the ciphertext primes.  The paper only defers to the HE
  security standard (Sec. 6.1, Table "mod-per-hamming-weight"); the reading
  used here is "the largest primes below 2^54 with q = 1 mod 2N, in
  descending order".
* ``primitive_root_2n``: psi = c^((q-1)/2N) for the smallest quadratic
  non-residue c mod q, so psi^N = c^((q-1)/2) = -1 and psi has order 2N.
* ``server_bin_bound``: the server maximum bin load mu when the paper gives no
  value: the least mu with b * P[Bin(k n, 1/b) >= mu] <= 2^-40 (a union bound
  over the b bins, one count on the conservative side).
"""
from __future__ import annotations

import math

T_PLAIN = 65537

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Miller-Rabin with the first twelve prime bases (deterministic below 3.3e24)."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def select_primes(n: int, count: int, bits: int = 54, skip: int = 0) -> list[int]:
    """The largest primes q < 2^bits with q = 1 mod 2n, descending; the first
    ``skip`` of them are passed over."""
    step = 2 * n
    q = ((1 << bits) - 1) // step * step + 1
    if q >= (1 << bits):
        q -= step
    out: list[int] = []
    while len(out) < skip + count:
        if is_prime(q):
            out.append(q)
        q -= step
    return out[skip:]


def smallest_nonresidue(q: int) -> int:
    c = 2
    while pow(c, (q - 1) // 2, q) != q - 1:
        c += 1
    return c


def primitive_root_2n(q: int, n: int) -> int:
    """psi with psi^n = -1 mod q (a primitive 2n-th root of unity)."""
    assert (q - 1) % (2 * n) == 0
    return pow(smallest_nonresidue(q), (q - 1) // (2 * n), q)


def code_length(lambda_bar: int, h: int) -> int:
    """Eq. (1): l(lambda_bar, h) = min{ l : C(l, h) >= 2^lambda_bar }.

    C(l, h) is increasing in l >= h, so the least l is found by bisection."""
    target = 1 << lambda_bar
    lo, hi = h, h
    while math.comb(hi, h) < target:
        lo, hi = hi, 2 * hi
    while lo < hi:                       # invariant: C(hi, h) >= target
        mid = (lo + hi) // 2
        if math.comb(mid, h) >= target:
            hi = mid
        else:
            lo = mid + 1
    return hi


def inv_factorial_mod_t(h: int, t: int = T_PLAIN) -> int:
    """(h!)^-1 mod t, the constant of Alg. 1."""
    return pow(math.factorial(h) % t, -1, t)


def server_bin_bound(n_items: int, n_bins: int, n_hash: int = 3, log2_fail: int = 40) -> int:
    """Least mu with  b * P[Bin(k n, 1/b) >= mu] <= 2^-log2_fail.

    The binomial tail is summed from its far end down (small terms first) in
    log-space floating point, which is ample to place the crossing."""
    trials = n_hash * n_items
    mean = trials / n_bins
    hi = min(trials, int(mean + 60 * math.sqrt(mean + 1) + 60))   # the pmf vanishes above `trials`

    def log_pmf(j: int) -> float:
        return (math.lgamma(trials + 1) - math.lgamma(j + 1) - math.lgamma(trials - j + 1)
                + j * math.log(1 / n_bins) + (trials - j) * math.log1p(-1 / n_bins))

    tail_ge = {}          # P[X >= j]
    acc = 0.0
    for j in range(hi, -1, -1):
        acc += math.exp(log_pmf(j))
        tail_ge[j] = acc
    limit = 2.0 ** -log2_fail
    mu = 0
    while n_bins * tail_ge.get(mu, 0.0) > limit:
        mu += 1
    return mu


# The paper's own server maximum bin loads (Tables "dipsi-cpsi", "cong-cpsi",
# "psisum-eval"), keyed by (n, b).
PAPER_MU = {
    (1 << 20, 8192): 526,
    (1 << 24, 8192): 6710,
    (1 << 28, 8192): 100565,
    (1 << 18, 16384): 100,
    (1 << 20, 16384): 296,
    (1 << 22, 16384): 976,
    (1 << 24, 16384): 3487,
}


def server_mu(n_items: int, n_bins: int) -> int:
    """The paper's value when it lists (n, b), else the 2^-40 bound."""
    return PAPER_MU.get((n_items, n_bins)) or server_bin_bound(n_items, n_bins)
