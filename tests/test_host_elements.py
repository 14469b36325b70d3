"""The library's host-side large-element calls against the oracle (no GPU needed): the element
length rule of Sec. 5 / Sec. 7 and the hashing of byte strings to lambda bits (SHA-256 of
FIPS 180-4, truncated), on empty, short, block-boundary and long elements."""
import numpy as np

from oracle import large as LG


def test_element_bits_rule():
    import paper_2310_14565_amd as pk
    for b, mc, ms in [(16384, 1, 100), (16384, 1, 296), (16384, 1, 976), (16384, 1, 3487), (8192, 1, 526),
                      (1024, 1, 11), (8, 1, 40), (1, 1, 1), (2, 3, 5)]:
        assert pk.large_element_bits(b, mc, ms) == LG.element_bits(b, mc, ms)
        assert pk.large_element_bits(b, mc, ms, 20) == LG.element_bits(b, mc, ms, 20)


def test_hash_elements_matches_sha256():
    import paper_2310_14565_amd as pk
    rng = np.random.default_rng(7)
    elems = [b"", b"abc", bytes(55), bytes(56), bytes(63), bytes(64), bytes(65), bytes(119), bytes(120),
             bytes(range(256)) * 5]
    elems += [bytes(rng.integers(0, 256, int(k), dtype=np.uint8)) for k in rng.integers(0, 300, 200)]
    for bits in (1, 7, 32, 49, 63, 64):
        got = pk.hash_elements(elems, bits)
        want = LG.hash_elements(elems, bits)
        assert (got == want).all(), bits
