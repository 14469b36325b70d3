"""Pins of the request and response compression in the oracle: ChaCha20 against the test
vectors of RFC 8439 (Sec. 2.1.1 quarter round, Sec. 2.3.2 block function), the expansion of a
seed into uniform polynomials against a direct Python rewrite of its definition, and
modulus switching against exact integer rounding and decryption."""
import numpy as np
import pytest

from oracle import params as P
from oracle.core import Context, chacha20_block, chacha_quarter
import workload as W


def test_rfc8439_quarter_round():
    assert chacha_quarter(0x11111111, 0x01020304, 0x9B8D6F43, 0x01234567) == \
        (0xEA2A92F4, 0xCB1CF8CE, 0x4581472E, 0x5881C4BB)


def test_rfc8439_block_function():
    key = np.frombuffer(bytes(range(32)), dtype="<u4")
    nonce = np.frombuffer(bytes([0, 0, 0, 9, 0, 0, 0, 0x4A, 0, 0, 0, 0]), dtype="<u4")
    out = chacha20_block(key, 1, nonce)
    want = [0xE4E7F110, 0x15593BD1, 0x1FDD0F50, 0xC47120A3, 0xC7F4D1C7, 0x0368C033, 0x9AAA2204,
            0x4E6CD4C3, 0x466482D2, 0x09AA9F07, 0x05D7C214, 0xA2028BD9, 0xD19C12B5, 0xB94E16DE,
            0xE883D0CB, 0x4E3C50A2]
    assert [int(x) for x in out] == want


def test_expansion_follows_its_definition():
    n = 1024
    ctx = Context(n, P.select_primes(n, 3))
    seed = bytes(W.rng(3, "seed").integers(0, 256, 32, dtype=np.uint8))
    a = ctx.expand_uniform(seed, 5, 2)
    key = np.frombuffer(seed, dtype="<u4")
    for jj, j in enumerate((5, 6)):
        for l, q in enumerate(ctx.primes):
            for k in (0, 1, 3, 4, 517, n - 1):
                blk = chacha20_block(key, k // 4, np.array([j, l, 0], np.uint32))
                w = blk[4 * (k % 4): 4 * (k % 4) + 4]
                W128 = int(w[0]) | int(w[1]) << 32 | int(w[2]) << 64 | int(w[3]) << 96
                assert int(a[jj, l, k]) == W128 % q
    assert (a < np.array(ctx.primes, dtype=np.uint64)[None, :, None]).all()
    # the same index gives the same polynomial, another index or seed another one
    assert (ctx.expand_uniform(seed, 6, 1)[0] == a[1]).all()
    assert (ctx.expand_uniform(seed, 7, 1)[0] != a[1]).mean() > 0.99
    # roughly uniform: the mean of a / q is near 1/2
    assert abs((a.astype(np.float64) / np.array(ctx.primes, dtype=np.float64)[None, :, None]).mean() - 0.5) < 0.01


@pytest.mark.parametrize("L", [2, 4])
def test_mod_switch_is_exact_rounding_and_decrypts(L):
    n = 1024
    ctx = Context(n, P.select_primes(n, L))
    ct = W.uniform_residues((2,), ctx.primes, n, 9, "ms")
    out = ctx.mod_switch(ct)
    Q, q0 = ctx.Q, ctx.primes[0]
    for comp in range(2):
        for k in (0, 1, 77, n - 1):
            x = ctx.residues_to_int([int(ct[comp, l, k]) for l in range(L)])
            if 2 * x > Q:
                x -= Q
            num = 2 * q0 * abs(x) + Q
            r = num // (2 * Q)
            r = -r if x < 0 else r
            assert int(out[comp, k]) == r % q0
    # a fresh encryption switched to q_0 still decrypts
    sk = W.secret_key(n, 10)
    m = W.rng(11, "m").integers(0, ctx.t, n, dtype=np.int64).astype(np.uint32)
    ct = ctx.encrypt(sk, ctx.encode(m), W.uniform_residues((), ctx.primes, n, 12, "enc-a"), W.errors(n, 12, "enc-e"))
    ctx0 = Context(n, [q0])
    assert (ctx0.decrypt_slots(sk, ctx.mod_switch(ct).reshape(2, 1, n)) == m).all()
