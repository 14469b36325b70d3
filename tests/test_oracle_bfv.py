"""Pins of the oracle's textbook FV against exact integer arithmetic and decryption."""
import math

import numpy as np
import pytest

from oracle.core import Context
import workload as W


def centred(x, m):
    x %= m
    return x - m if 2 * x > m else x


def negacyclic(a, b):
    n = len(a)
    c = [0] * n
    for i in range(n):
        for j in range(n):
            if i + j < n:
                c[i + j] += a[i] * b[j]
            else:
                c[i + j - n] -= a[i] * b[j]
    return c


def as_ints(ctx, ct, comp):
    return ctx.poly_to_ints(np.asarray(ct)[comp])


def setup(n, L, seed=1):
    ctx = Context.standard(n, L)
    sk = W.secret_key(n, seed)
    return ctx, sk


def enc(ctx, sk, slots, seed):
    a = W.uniform_residues((), ctx.primes, ctx.n, seed, "a")
    e = W.errors((ctx.n,), seed, "e")
    return ctx.encrypt(sk, ctx.encode(slots), a, e), a, e


def rand_slots(n, seed, hi=65537):
    return W.rng(seed, "slots").integers(0, hi, size=n).astype(np.uint32)


def test_modulus_is_odd_and_coprime_to_t():
    for n, L in [(4096, 2), (8192, 4), (16384, 8)]:
        ctx = Context.standard(n, L)
        assert ctx.Q % 2 == 1 and math.gcd(ctx.Q, ctx.t) == 1   # rounding ties are impossible


@pytest.mark.parametrize("n,L", [(16, 2), (32, 3)])
def test_encryption_phase_identity(n, L):
    """c0 + c1*s = Delta*[m]_t - e  (mod Q), checked with Python integers."""
    ctx, sk = setup(n, L)
    slots = rand_slots(n, 4)
    ct, a, e = enc(ctx, sk, slots, 5)
    m = ctx.encode(slots)
    c0, c1 = as_ints(ctx, ct, 0), as_ints(ctx, ct, 1)
    assert c1 == ctx.poly_to_ints(a)
    s = [int(v) for v in sk]
    c1s = negacyclic(c1, s)
    for i in range(n):
        want = ctx.delta * centred(int(m[i]), ctx.t) - int(e[i])
        assert (c0[i] + c1s[i] - want) % ctx.Q == 0


@pytest.mark.parametrize("n,L", [(64, 2), (4096, 2), (8192, 4)])
def test_decrypt_encrypt(n, L):
    ctx, sk = setup(n, L)
    slots = rand_slots(n, 6)
    ct, _, _ = enc(ctx, sk, slots, 7)
    assert (ctx.decrypt_slots(sk, ct) == slots).all()
    assert ctx.noise_budget(sk, ct) > 0


def test_decrypt_and_budget_of_hand_made_ciphertexts():
    n, L = 16, 2
    ctx, sk = setup(n, L)
    m = rand_slots(n, 8)
    for v in (0, 1, -1, ctx.delta // 4, -(ctx.delta // 4), 12345):
        c0 = [(ctx.delta * centred(int(x), ctx.t) + v) % ctx.Q for x in m]
        ct = np.stack([ctx.ints_to_poly(c0), ctx.ints_to_poly([0] * n)])
        assert (ctx.decrypt_poly(sk, ct) == m).all()
        worst = max(abs(centred(ctx.t * c, ctx.Q)) for c in c0)
        assert ctx.noise_budget(sk, ct) == ctx.Q.bit_length() - worst.bit_length() - 1


def test_plain_multiply_and_constants():
    n, L = 64, 2
    ctx, sk = setup(n, L)
    x, y = rand_slots(n, 9), rand_slots(n, 10)
    ct, _, _ = enc(ctx, sk, x, 11)
    t = ctx.t
    pm = ctx.mul_plain(ct, ctx.encode(y))
    assert (ctx.decrypt_slots(sk, pm) == x.astype(np.int64) * y % t).all()
    ac = ctx.add_plain_const(ct, t - 3)
    assert (ctx.decrypt_slots(sk, ac) == (x.astype(np.int64) - 3) % t).all()
    ap = ctx.add_plain(ct, ctx.encode(y))
    assert (ctx.decrypt_slots(sk, ap) == (x.astype(np.int64) + y) % t).all()
    mc = ctx.mul_const(ct, 19115)
    assert (ctx.decrypt_slots(sk, mc) == x.astype(np.int64) * 19115 % t).all()
    # the plaintext product is (c0*p, c1*p) with p the centred lift of the encoding
    p = [centred(int(v), t) for v in ctx.encode(y)]
    for comp in (0, 1):
        want = [v % ctx.Q for v in negacyclic(as_ints(ctx, ct, comp), p)]
        assert as_ints(ctx, pm, comp) == want


@pytest.mark.parametrize("n,L", [(16, 2), (16, 3), (32, 4)])
def test_multiply_is_the_textbook_rounding(n, L):
    """out_k = [round(t/Q * (x (x) y)_k)]_Q on centred lifts, with Python integers."""
    ctx, sk = setup(n, L)
    cx, _, _ = enc(ctx, sk, rand_slots(n, 12), 13)
    cy, _, _ = enc(ctx, sk, rand_slots(n, 14), 15)
    got = ctx.multiply(cx, cy)
    Q, t = ctx.Q, ctx.t
    X = [[centred(v, Q) for v in as_ints(ctx, cx, c)] for c in (0, 1)]
    Y = [[centred(v, Q) for v in as_ints(ctx, cy, c)] for c in (0, 1)]
    d0 = negacyclic(X[0], Y[0])
    d1 = [u + v for u, v in zip(negacyclic(X[0], Y[1]), negacyclic(X[1], Y[0]))]
    d2 = negacyclic(X[1], Y[1])
    for comp, d in enumerate((d0, d1, d2)):
        want = [((2 * t * v + Q) // (2 * Q)) % Q for v in d]   # floor(t v / Q + 1/2)
        assert as_ints(ctx, got, comp) == want


@pytest.mark.parametrize("n,L", [(32, 2), (64, 3)])
def test_relinearisation_key_identity(n, L):
    """(c0' + c1' s) - (d0 + d1 s + d2 s^2) = -sum_i D_i e_i (mod Q), D_i the gadget digits."""
    ctx, sk = setup(n, L)
    ka = W.uniform_residues((L,), ctx.primes, n, 20, "rlk-a")
    ke = W.errors((L, n), 21, "rlk-e")
    rlk = ctx.keygen_relin(sk, ka, ke)
    cx, _, _ = enc(ctx, sk, rand_slots(n, 16), 17)
    cy, _, _ = enc(ctx, sk, rand_slots(n, 18), 19)
    d = ctx.multiply(cx, cy)
    r = ctx.relin(d, rlk)
    s = [int(v) for v in sk]
    s2 = negacyclic(s, s)
    D = [[int(v) * pow(ctx.Q // q, -1, q) % q for v in d[2, i]] for i, q in enumerate(ctx.primes)]
    noise = [0] * n
    for i in range(L):
        for k, v in enumerate(negacyclic(D[i], [int(x) for x in ke[i]])):
            noise[k] -= v
    lhs = [u + v for u, v in zip(as_ints(ctx, r, 0), negacyclic(as_ints(ctx, r, 1), s))]
    d0, d1, d2 = (as_ints(ctx, d, c) for c in range(3))
    rhs = [u + v + w for u, v, w in zip(d0, negacyclic(d1, s), negacyclic(d2, s2))]
    for k in range(n):
        assert (lhs[k] - rhs[k] - noise[k]) % ctx.Q == 0
    # and the key itself: rlk_i0 + rlk_i1 s = (Q/q_i) s^2 - e_i
    for i, q in enumerate(ctx.primes):
        k0 = ctx.poly_to_ints(rlk[i, 0])
        k1s = negacyclic(ctx.poly_to_ints(rlk[i, 1]), s)
        for k in range(n):
            assert (k0[k] + k1s[k] - (ctx.Q // q) * s2[k] + int(ke[i, k])) % ctx.Q == 0


@pytest.mark.parametrize("n,L", [(64, 2), (4096, 2)])
def test_multiply_relin_decrypts(n, L):
    ctx, sk = setup(n, L)
    rlk = ctx.keygen_relin(sk, W.uniform_residues((L,), ctx.primes, n, 30, "rlk-a"),
                           W.errors((L, n), 31, "rlk-e"))
    x, y = rand_slots(n, 32), rand_slots(n, 33)
    cx, _, _ = enc(ctx, sk, x, 34)
    cy, _, _ = enc(ctx, sk, y, 35)
    r = ctx.relin(ctx.multiply(cx, cy), rlk)
    assert (ctx.decrypt_slots(sk, r) == x.astype(np.int64) * y % ctx.t).all()
    assert ctx.noise_budget(sk, r) > 0
