"""Seeded synthetic inputs for PEPSI PSI-cardinality.

The ONLY module shared by the GPU library's harness and the reference
oracle.  It draws random numbers and nothing else: no part of the scheme's
arithmetic lives here.  Every draw is a pure function of (seed, tag).

Input recipe (the paper's 32-bit setting, Sec. 7: random 32-bit identifiers):
  * server set: n distinct uniform ``bits``-bit integers;
  * client set: ``planted`` elements drawn without replacement from the server
    set plus m - planted distinct uniform elements outside it, shuffled;
  * secret key: uniform ternary {-1, 0, 1}^N;
  * encryption / key randomness: uniform residues a in [0, q_l) per limb and
    errors e from a rounded Gaussian of sigma 3.2 clipped at 6 sigma;
  * output mask: N uniform values in [0, t) with the last one fixing the sum
    to 0 mod t (Alg. 5).
"""
from __future__ import annotations

import zlib

import numpy as np

SIGMA = 3.2
CLIP = 19  # ceil(6 sigma)


def rng(seed: int, tag: str) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed & 0xFFFFFFFF, seed >> 32, zlib.crc32(tag.encode())])))


def server_items(n: int, bits: int, seed: int) -> np.ndarray:
    g = rng(seed, "server-set")
    space = 1 << bits
    if n > space:
        raise ValueError("set larger than the element space")
    if n * 4 > space:
        return g.permutation(space)[:n].astype(np.uint32)
    out = np.unique(g.integers(0, space, size=int(n * 1.1) + 16, dtype=np.uint64))
    while out.shape[0] < n:
        out = np.unique(np.concatenate([out, g.integers(0, space, size=n, dtype=np.uint64)]))
    return g.permutation(out)[:n].astype(np.uint32)


def client_items(m: int, server: np.ndarray, planted: int, bits: int, seed: int) -> np.ndarray:
    g = rng(seed, "client-set")
    common = g.choice(server, size=planted, replace=False).astype(np.uint64)
    server_set = set(int(x) for x in server) if server.shape[0] <= (1 << 16) else None
    srt = np.sort(server.astype(np.uint64))
    others: list[int] = []
    seen = set(int(x) for x in common)
    while len(others) < m - planted:
        x = int(g.integers(0, 1 << bits, dtype=np.uint64))
        if x in seen:
            continue
        inside = (x in server_set) if server_set is not None else \
            (np.searchsorted(srt, x) < srt.shape[0] and srt[np.searchsorted(srt, x)] == x)
        if inside:
            continue
        seen.add(x)
        others.append(x)
    out = np.concatenate([common, np.array(others, dtype=np.uint64)])
    return g.permutation(out).astype(np.uint32)


def secret_key(n: int, seed: int) -> np.ndarray:
    return (rng(seed, "secret-key").integers(0, 3, size=n) - 1).astype(np.int8)


def uniform_residues(shape_prefix, primes, n: int, seed: int, tag: str) -> np.ndarray:
    """uint64 array of shape (*shape_prefix, L, n); limb l uniform in [0, q_l)."""
    g = rng(seed, tag)
    shape_prefix = tuple(shape_prefix)
    out = np.empty(shape_prefix + (len(primes), n), dtype=np.uint64)
    for l, q in enumerate(primes):
        out[..., l, :] = g.integers(0, int(q), size=shape_prefix + (n,), dtype=np.uint64)
    return out


def errors(shape, seed: int, tag: str) -> np.ndarray:
    g = rng(seed, tag)
    e = np.rint(g.normal(0.0, SIGMA, size=shape))
    return np.clip(e, -CLIP, CLIP).astype(np.int32)


def zero_sum_mask(n: int, t: int, seed: int) -> np.ndarray:
    g = rng(seed, "mask")
    r = g.integers(0, t, size=n, dtype=np.int64)
    r[-1] = (-int(r[:-1].sum())) % t
    return r.astype(np.uint32)


def planes_random(count: int, n: int, seed: int, tag: str = "planes") -> np.ndarray:
    """Random 0/1 slot vectors (used for kernel-level checks)."""
    return rng(seed, tag).integers(0, 2, size=(count, n), dtype=np.uint32)


def item_values(n: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """Server values (PSI-Sum) or labels (labelled PSI): n uniform integers in [lo, hi)."""
    return rng(seed, "item-values").integers(lo, hi, size=n, dtype=np.int64).astype(np.uint32)


def byte_elements(n: int, length: int, seed: int, tag: str = "byte-elements") -> np.ndarray:
    """Large elements (Sec. 7: strings such as credentials or 256-bit strings): n distinct
    uniform byte strings of the given length, as the rows of a uint8 [n][length] array."""
    g = rng(seed, tag)
    out = g.integers(0, 256, size=(n, length), dtype=np.uint8)
    if length < 16:                 # beyond 16 bytes a repeat has probability below 2^-88
        _, first = np.unique(out, axis=0, return_index=True)
        if first.shape[0] != n:
            raise ValueError("repeated element; use longer elements")
    return out
