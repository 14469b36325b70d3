"""Pins of constant-weight encoding and hashing to bins."""
import itertools
import math

import numpy as np
import pytest

from oracle import cw, hashing
from oracle import params as P
import workload as W


@pytest.mark.parametrize("ell,h", [(6, 1), (7, 2), (9, 3), (10, 4), (12, 5)])
def test_cw_is_a_bijection_onto_weight_h_words(ell, h):
    words = set()
    for v in range(math.comb(ell, h)):
        pos = cw.encode_one(v, ell, h)
        assert len(set(pos)) == h and all(0 <= p < ell for p in pos)
        words.add(tuple(sorted(pos)))
    assert words == set(itertools.combinations(range(ell), h))


def test_cw_vectorised_matches_scalar():
    rng = np.random.default_rng(0)
    for ell, h, bits in [(569, 4, 32), (363, 2, 16), (24, 8, 19)]:
        v = rng.integers(0, 1 << bits, size=300, dtype=np.int64)
        v = np.concatenate([v, [0, (1 << bits) - 1]])
        got = cw.encode_many(v, ell, h)
        for x, row in zip(v, got):
            assert list(row) == cw.encode_one(int(x), ell, h)


def test_cw_range_checked():
    with pytest.raises(ValueError):
        cw.encode_one(math.comb(10, 3), 10, 3)


def test_planes_weight_and_dummy():
    pos = np.array([[5, 2], [cw.NO_POS, cw.NO_POS], [1, 0]], dtype=np.uint16)
    pl = cw.planes(pos, 7)
    assert pl.shape == (7, 3)
    assert pl[:, 0].sum() == 2 and pl[5, 0] == 1 and pl[2, 0] == 1
    assert pl[:, 1].sum() == 0                  # dummy -> all-zero word (Sec. 4.1)


def test_mix64_splitmix_reference_output():
    # SplitMix64 seeded with 0 outputs mix64(0x9E3779B97F4A7C15) first.
    assert hashing.mix64(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF


def test_vectorised_hash_matches_scalar():
    xs = np.array([0, 1, 2, 0xFFFFFFFF, 123456789], dtype=np.uint64)
    for i in (1, 2, 3):
        got = hashing.bins_of_array(xs, i, 99, 8192)
        assert list(got) == [hashing.bin_of(int(x), i, 99, 8192) for x in xs]


def test_cuckoo_places_every_item_once_in_one_of_its_bins():
    items = W.server_items(1024, 32, 5)
    table, valid = hashing.cuckoo_table(items, 8192, 77)
    assert valid.sum() == 1024
    placed = table[valid.astype(bool)]
    assert sorted(placed.tolist()) == sorted(items.tolist())
    for k in np.nonzero(valid)[0]:
        x = int(table[k])
        assert k in {hashing.bin_of(x, i, 77, 8192) for i in (1, 2, 3)}


def test_cuckoo_failure_is_an_error():
    with pytest.raises(hashing.CuckooFailure):
        hashing.cuckoo_table(list(range(40)), 16, 3)          # m > b cannot fit
    with pytest.raises(ValueError):
        hashing.cuckoo_table([1, 1], 16, 3)


def test_simple_hashing_bins_and_order():
    items = W.server_items(3000, 32, 6)
    table, valid, max_load = hashing.simple_table(items, 256, 64, 9)
    where = {}
    for ip in range(64):
        for k in range(256):
            if valid[ip, k]:
                where.setdefault(int(table[ip, k]), []).append((k, ip))
    index = {int(x): n for n, x in enumerate(items)}
    for x in items.tolist():
        want = {hashing.bin_of(x, i, 9, 256) for i in (1, 2, 3)}
        assert sorted(k for k, _ in where[x]) == sorted(want)     # each distinct bin, once
    for k in range(256):                                           # input order within a bin
        col = [index[int(v)] for v, ok in zip(table[:, k], valid[:, k]) if ok]
        assert col == sorted(col)
        assert all(valid[len(col):, k] == 0)
    assert max_load == int(valid.sum(axis=0).max())


def test_bin_overflow_is_an_error():
    items = W.server_items(3000, 32, 6)
    _, _, max_load = hashing.simple_table(items, 256, 64, 9)
    with pytest.raises(hashing.BinOverflow):
        hashing.simple_table(items, 256, max_load - 1, 9)


def test_observed_load_below_paper_mu():
    """Paper-sized check (Table 'dipsi-cpsi'): n = 2^20, b = 8192 stays within mu = 526."""
    items = W.server_items(1 << 20, 32, 2024)
    _, _, max_load = hashing.simple_table(items, 8192, P.server_mu(1 << 20, 8192), 0x5EED)
    assert max_load <= 526
