"""Oracle (test infrastructure only): hashing to bins (Sec. 3.3, Sec. 4.1, Alg. 6).

The paper names cuckoo hashing with k = 3 hash functions and no stash for the
client and appends every server element to the bins "chosen by the binning
strategy".  It does not fix the hash functions; the reading used here is

    H_i(x) = mix64(x XOR (seed + i * 0x9E3779B97F4A7C15 mod 2^64)) mod b,  i = 1..k,

where mix64 is the SplitMix64 output finaliser (Steele, Lea, Flood 2014):
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31.

Cuckoo insertion (Sec. 3.3): x goes to bin H_1(x); an occupant x' that sat
in its bin H_i(x') is evicted and moves on to H_{(i mod k)+1}(x'); more than
``max_evictions`` evictions for one insertion is a protocol failure (no stash).
Server simple hashing: y is appended to each DISTINCT bin among H_1..H_k(y),
elements in input order; a bin holding more than mu elements is a failure.

Permutation-based hashing (PBH, Sec. 3.3) with b = 2^c bins and lambda-bit
elements x = x_H || x_L (|x_H| = c): hash function i puts x into bin
x_H XOR H_i(x_L) and stores the shorter value (i - 1) 2^(lambda - c) + x_L.  The
paper's description has one hash function; with k of them the stored value must
also name i, or x placed by H_i and a different y placed by H_j could meet in a
bin with x_L = y_L.  Equal stored values in equal bins then imply equal
elements.  The server stores all k (bin, value) entries of an element (entries
of one element never share a value, so none is dropped and none can match twice).
"""
from __future__ import annotations

import numpy as np

GOLDEN = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


class CuckooFailure(Exception):
    pass


class BinOverflow(Exception):
    pass


def mix64(z: int) -> int:
    z &= M64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & M64
    z ^= z >> 31
    return z


def bin_of(x: int, i: int, seed: int, n_bins: int) -> int:
    """H_i(x) for i in 1..k."""
    return mix64(x ^ ((seed + i * GOLDEN) & M64)) % n_bins


def bins_of_array(xs: np.ndarray, i: int, seed: int, n_bins: int) -> np.ndarray:
    """H_i over a numpy array (uint64 wrap-around arithmetic is exact mod 2^64)."""
    z = xs.astype(np.uint64) ^ np.uint64((seed + i * GOLDEN) & M64)
    z ^= z >> np.uint64(30)
    z *= np.uint64(0xBF58476D1CE4E5B9)
    z ^= z >> np.uint64(27)
    z *= np.uint64(0x94D049BB133111EB)
    z ^= z >> np.uint64(31)
    return (z % np.uint64(n_bins)).astype(np.int64)


def pbh_place(x: int, i: int, seed: int, n_bins: int, lam: int):
    """PBH: (bin, stored value) of element x under hash function i (b = n_bins = 2^c)."""
    c = n_bins.bit_length() - 1
    assert n_bins == 1 << c and lam > c
    low = lam - c
    xh, xl = x >> low, x & ((1 << low) - 1)
    return xh ^ bin_of(xl, i, seed, n_bins), ((i - 1) << low) | xl


def cuckoo_table(items, n_bins: int, seed: int, n_hash: int = 3, max_evictions: int = 500,
                 pbh_bits: int | None = None):
    """Client table T_c (gamma = 1): returns (table uint32[b], valid uint8[b]; uint64 once a value
    exceeds 32 bits).  With pbh_bits (the element length lambda) the table holds PBH values
    instead of the elements."""
    items = [int(x) for x in items]
    if len(set(items)) != len(items):
        raise ValueError("duplicate client items")
    table = [None] * n_bins
    which = [0] * n_bins
    for x in items:
        cur, idx, evictions = x, 1, 0
        while True:
            if pbh_bits:
                pos = pbh_place(cur, idx, seed, n_bins, pbh_bits)[0]
            else:
                pos = bin_of(cur, idx, seed, n_bins)
            if table[pos] is None:
                table[pos], which[pos] = cur, idx
                break
            # evict the occupant; it moves on to its next hash function
            evicted, evicted_idx = table[pos], which[pos]
            table[pos], which[pos] = cur, idx
            cur, idx = evicted, evicted_idx % n_hash + 1
            evictions += 1
            if evictions > max_evictions:
                raise CuckooFailure(f"eviction limit {max_evictions} reached")
    stored = [0] * n_bins
    valid = np.zeros(n_bins, dtype=np.uint8)
    for k, v in enumerate(table):
        if v is not None:
            stored[k] = pbh_place(v, which[k], seed, n_bins, pbh_bits)[1] if pbh_bits else v
            valid[k] = 1
    return np.array(stored, dtype=_value_dtype(max(stored, default=0))), valid


def _value_dtype(largest: int):
    """uint32 tables for values of up to 32 bits (the 32-bit elements), uint64 beyond."""
    return np.uint32 if largest < (1 << 32) else np.uint64


def simple_table(items: np.ndarray, n_bins: int, mu: int, seed: int, n_hash: int = 3,
                 pbh_bits: int | None = None, with_index: bool = False):
    """Server table T_s: returns (table uint32[mu][b] (uint64 once a value exceeds 32 bits),
    valid uint8[mu][b], max_load), and with
    with_index also the element's input position per entry (int64[mu][b], -1 for dummies).

    Entry (i', k) is the i'-th element appended to bin k, in input order.  With pbh_bits the
    entries are PBH values, one per hash function (in hash-function order within an element)."""
    items = np.asarray(items, dtype=np.uint64)
    n = items.shape[0]
    elem = np.broadcast_to(np.arange(n), (n_hash, n))
    if pbh_bits:
        c = n_bins.bit_length() - 1
        assert n_bins == 1 << c and pbh_bits > c
        low = pbh_bits - c
        xh = items >> np.uint64(low)
        xl = items & np.uint64((1 << low) - 1)
        h = np.stack([(xh ^ bins_of_array(xl, i, seed, n_bins).astype(np.uint64)).astype(np.int64)
                      for i in range(1, n_hash + 1)])                                    # [k][n]
        vals = np.stack([(np.uint64(i - 1) << np.uint64(low)) | xl for i in range(1, n_hash + 1)])
        keep = np.ones_like(h, dtype=bool)
    else:
        h = np.stack([bins_of_array(items, i, seed, n_bins) for i in range(1, n_hash + 1)])  # [k][n]
        vals = np.broadcast_to(items, (n_hash, n))
        # distinct bins of each element: drop H_i(y) equal to an earlier H_j(y)
        keep = np.ones_like(h, dtype=bool)
        for i in range(1, n_hash):
            for j in range(i):
                keep[i] &= h[i] != h[j]
    fn = np.broadcast_to(np.arange(n_hash)[:, None], (n_hash, n))
    sel_bin, sel_elem, sel_fn, sel_val = h[keep], elem[keep], fn[keep], vals[keep]
    # input order within each bin: stable sort by (bin, element index, hash function)
    order = np.lexsort((sel_fn, sel_elem, sel_bin))
    sel_bin, sel_elem, sel_val = sel_bin[order], sel_elem[order], sel_val[order]
    counts = np.bincount(sel_bin, minlength=n_bins)
    max_load = int(counts.max()) if counts.size else 0
    if max_load > mu:
        raise BinOverflow(f"server bin load {max_load} exceeds mu={mu}")
    starts = np.concatenate([[0], np.cumsum(counts)[:-1]])
    rank = np.arange(sel_bin.shape[0]) - starts[sel_bin]
    dt = _value_dtype(int(sel_val.max()) if sel_val.size else 0)
    table = np.zeros((mu, n_bins), dtype=dt)
    valid = np.zeros((mu, n_bins), dtype=np.uint8)
    table[rank, sel_bin] = sel_val.astype(dt)
    valid[rank, sel_bin] = 1
    if with_index:
        index = np.full((mu, n_bins), -1, dtype=np.int64)
        index[rank, sel_bin] = sel_elem
        return table, valid, max_load, index
    return table, valid, max_load
