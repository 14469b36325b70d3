"""Pins of the oracle's negacyclic arithmetic and batching against definitions."""
import numpy as np
import pytest

from oracle import params as P
from oracle.core import Context, lib
import workload as W


def brv(k, bits):
    return int(format(k, f"0{bits}b")[::-1], 2) if bits else 0


@pytest.mark.parametrize("n", [1, 2, 4, 16, 64, 256])
def test_eval_fwd_is_evaluation_at_roots(n):
    q = P.select_primes(max(n, 2), 1)[0]
    psi = P.primitive_root_2n(q, n) if n > 1 else q - 1
    a = W.uniform_residues((), [q], n, n, "a")[0]
    got = a.copy()
    lib().or_eval_fwd(got, n, q, psi)
    for k in range(n):
        x = pow(psi, 2 * k + 1, q)
        assert int(got[k]) == sum(int(c) * pow(x, i, q) for i, c in enumerate(a)) % q
        assert x != 1 and pow(x, n, q) == q - 1           # a root of X^n + 1
    back = got.copy()
    lib().or_eval_inv(back, n, q, psi)
    assert (back == a).all()


@pytest.mark.parametrize("n", [4096, 16384])
def test_eval_fwd_sampled_points_large(n):
    q = P.select_primes(n, 1)[0]
    psi = P.primitive_root_2n(q, n)
    a = W.uniform_residues((), [q], n, 3, "a")[0]
    got = a.copy()
    lib().or_eval_fwd(got, n, q, psi)
    for k in (0, 1, n // 2, n - 1, 1234 % n):
        assert int(got[k]) == lib().or_poly_eval_point(a, n, q, pow(psi, 2 * k + 1, q))
    back = got.copy()
    lib().or_eval_inv(back, n, q, psi)
    assert (back == a).all()


@pytest.mark.parametrize("n", [8, 32, 128])
def test_products_agree_and_are_ring_products(n):
    q = P.select_primes(n, 1)[0]
    psi = P.primitive_root_2n(q, n)
    a = W.uniform_residues((), [q], n, 1, "a")[0]
    b = W.uniform_residues((), [q], n, 2, "b")[0]
    c1 = np.zeros(n, np.uint64)
    c2 = np.zeros(n, np.uint64)
    lib().or_poly_mul_schoolbook(a, b, c1, n, q)
    lib().or_poly_mul_eval(a, b, c2, n, q, psi)
    assert (c1 == c2).all()
    # the product modulo X^n + 1 is the product of evaluations at each root of X^n + 1
    for k in range(0, n, max(1, n // 8)):
        x = pow(psi, 2 * k + 1, q)
        ev = lambda p: lib().or_poly_eval_point(np.ascontiguousarray(p), n, q, x)
        assert ev(c1) == ev(a) * ev(b) % q
    # X * X^(n-1) = X^n = -1
    e1 = np.zeros(n, np.uint64); e1[1] = 1
    en = np.zeros(n, np.uint64); en[n - 1] = 1
    lib().or_poly_mul_schoolbook(e1, en, c1, n, q)
    assert c1[0] == q - 1 and not c1[1:].any()


@pytest.mark.parametrize("n", [16, 256, 4096])
def test_batching(n):
    ctx = Context.standard(n, 1)
    t = ctx.t
    y1 = W.rng(1, "y1").integers(0, t, size=n).astype(np.uint32)
    y2 = W.rng(2, "y2").integers(0, t, size=n).astype(np.uint32)
    p1, p2 = ctx.encode(y1), ctx.encode(y2)
    assert (ctx.decode(p1) == y1).all()
    # slot k is the value at psi_t^(2k+1) (natural order)
    for k in (0, 1, n - 1):
        x = pow(ctx.psi_t, 2 * k + 1, t)
        assert sum(int(c) * pow(x, i, t) for i, c in enumerate(p1)) % t == y1[k]
    # products of encodings decode to slot-wise products (batching is a ring isomorphism)
    prod = np.zeros(n, np.uint64)
    lib().or_poly_mul_eval(p1.astype(np.uint64), p2.astype(np.uint64), prod, n, t, ctx.psi_t)
    assert (ctx.decode(prod.astype(np.uint32)) == (y1.astype(np.int64) * y2 % t)).all()
