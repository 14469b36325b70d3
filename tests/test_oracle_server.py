"""Pins of the oracle's server computation (Alg. 1, Alg. 2, Alg. 4, Alg. 5)."""
import itertools
import math

import numpy as np
import pytest

from oracle import cw, params as P, protocol as PR
from oracle.core import Context
import workload as W


@pytest.mark.parametrize("ell,h", [(5, 2), (6, 3), (7, 4), (5, 1)])
def test_arith_cw_eq_truth_table_plaintext(ell, h):
    """Alg. 1 in Z_t: e = (1/h!) prod_{r<h} (h' - r) is 1 iff the codewords are equal, else 0."""
    t = P.T_PLAIN
    k = P.inv_factorial_mod_t(h)
    words = list(itertools.combinations(range(ell), h))
    for x in words:
        for y in words:
            hp = len(set(x) & set(y))               # h' = sum_j x_j y_j
            e = k
            for r in range(h):
                e = e * (hp - r) % t
            assert e == (1 if x == y else 0)
    # a dummy (all-zero word) never matches
    e = k
    for r in range(h):
        e = e * (0 - r) % t
    assert e == 0


def small_keys(ctx, seed):
    sk = W.secret_key(ctx.n, seed)
    rlk = ctx.keygen_relin(sk, W.uniform_residues((ctx.L,), ctx.primes, ctx.n, seed, "rlk-a"),
                           W.errors((ctx.L, ctx.n), seed, "rlk-e"))
    return sk, rlk


def encrypt_planes(ctx, sk, planes, seed):
    ell = planes.shape[0]
    return PR.encrypt_planes(ctx, sk, planes,
                             W.uniform_residues((ell,), ctx.primes, ctx.n, seed, "enc-a"),
                             W.errors((ell, ctx.n), seed, "enc-e"))


@pytest.mark.parametrize("ell,h", [(5, 2), (6, 3)])
def test_arith_cw_eq_encrypted_every_pair(ell, h):
    """Alg. 1 through encryption: every (client, server) codeword pair, one pair per slot."""
    n = 16
    ctx = Context.standard(n, 3)
    sk, rlk = small_keys(ctx, 40)
    words = list(itertools.combinations(range(ell), h)) + [None]     # None = dummy
    pairs = list(itertools.product(words, words))
    k = P.inv_factorial_mod_t(h)
    for start in range(0, len(pairs), n):
        chunk = pairs[start:start + n]
        cpos = np.full((n, h), cw.NO_POS, np.uint16)
        spos = np.full((1, n, h), cw.NO_POS, np.uint16)
        for slot, (x, y) in enumerate(chunk):
            if x is not None:
                cpos[slot] = x
            if y is not None:
                spos[0, slot] = y
        cts = encrypt_planes(ctx, sk, cw.planes(cpos, ell), 41 + start)
        out = ctx.server_eval(cts, spos, rlk, h, mask=None, finalize=True)
        got = ctx.decrypt_slots(sk, out)
        for slot, (x, y) in enumerate(chunk):
            assert got[slot] == (1 if (x is not None and x == y) else 0)
        # the product tree before the 1/h! factor decrypts to h! * [x == y]
        raw = ctx.server_eval(cts, spos, rlk, h, mask=None, finalize=False)
        got_raw = ctx.decrypt_slots(sk, raw)
        for slot, (x, y) in enumerate(chunk):
            assert got_raw[slot] * k % ctx.t == got[slot]


def test_select_sum_is_the_sum_of_plain_products():
    n, ell, h = 32, 9, 3
    ctx = Context.standard(n, 2)
    sk, _ = small_keys(ctx, 50)
    cpos = cw.encode_many(W.rng(51, "c").integers(0, math.comb(ell, h), n), ell, h)
    spos = cw.encode_many(W.rng(52, "s").integers(0, math.comb(ell, h), n), ell, h)
    spos[3] = cw.NO_POS
    cts = encrypt_planes(ctx, sk, cw.planes(cpos, ell), 53)
    got = ctx.select_sum(cts, spos, h)
    want = ctx.zeros_ct()
    planes = cw.planes(spos, ell)
    for j in range(ell):
        pm = ctx.mul_plain(cts[j], ctx.encode(planes[j]))
        for l, q in enumerate(ctx.primes):
            want[:, l] = (want[:, l].astype(object) + pm[:, l].astype(object)) % q
    assert (got == want).all()
    # decrypts to h' = |cw(x) & cw(y)| per slot
    hp = ctx.decrypt_slots(sk, got)
    for k in range(n):
        expect = 0 if k == 3 else len(set(cpos[k]) & set(spos[k]))
        assert hp[k] == expect


def test_mask_and_finalize_are_linear():
    """Applying (h!)^-1 and the mask after the sum equals the definition term by term."""
    n, ell, h = 16, 6, 2
    ctx = Context.standard(n, 2)
    sk, rlk = small_keys(ctx, 60)
    cpos = cw.encode_many(W.rng(61, "c").integers(0, math.comb(ell, h), n), ell, h)
    spos = cw.encode_many(W.rng(62, "s").integers(0, math.comb(ell, h), 3 * n), ell, h).reshape(3, n, h)
    cts = encrypt_planes(ctx, sk, cw.planes(cpos, ell), 63)
    mask = W.zero_sum_mask(n, ctx.t, 64)
    out = ctx.server_eval(cts, spos, rlk, h, mask=mask)
    acc = ctx.zeros_ct()
    for ip in range(3):
        e = ctx.server_batch(cts, spos[ip], rlk, h)
        for l, q in enumerate(ctx.primes):
            acc[:, l] = (acc[:, l].astype(object) + e[:, l].astype(object)) % q
    want = ctx.add_plain(ctx.mul_const(acc, P.inv_factorial_mod_t(h)), ctx.encode(mask))
    assert (out == want).all()
    part = ctx.server_eval(cts, spos, rlk, h, finalize=False, begin=1, end=3)
    e0 = ctx.server_batch(cts, spos[0], rlk, h)
    for l, q in enumerate(ctx.primes):
        assert ((part[:, l].astype(object) + e0[:, l].astype(object)) % q == acc[:, l]).all()


@pytest.mark.parametrize("seed", [1, 2])
def test_small_psi_cardinality_and_indicator(seed):
    cfg = PR.Config(n=64, L=3, h=2, item_bits=8, mu=0)
    server = W.server_items(60, 8, seed)
    cfg.mu = P.server_bin_bound(60, 64)
    client = W.client_items(20, server, 7, 8, seed + 100)
    ctx = Context.standard(cfg.n, cfg.L)
    sk, rlk = small_keys(ctx, seed + 200)
    ctab, cval, _, planes = PR.client_prepare(cfg, client)
    stab, sval, spos, _ = PR.server_prepare(cfg, server)
    cts = encrypt_planes(ctx, sk, planes, seed + 300)
    mask = W.zero_sum_mask(cfg.n, ctx.t, seed + 400)
    card = ctx.server_eval(cts, spos, rlk, cfg.h, mask=mask)
    slots = ctx.decrypt_slots(sk, card)
    assert PR.extract_cardinality(slots) == len(set(client.tolist()) & set(server.tolist())) == 7
    ind = ctx.decrypt_slots(sk, ctx.server_eval(cts, spos, rlk, cfg.h))
    assert (ind == PR.plaintext_membership(ctab, cval, stab, sval)).all()


@pytest.mark.parametrize("seed", [3, 4])
def test_small_psi_sum_and_labels(seed):
    """Alg. 5 (PSI-Sum, masked) and Alg. 4 (labelled PSI) against their plaintext meaning, and
    unit values reproduce the PSI-cardinality ciphertext (Sec. 5.3)."""
    cfg = PR.Config(n=64, L=3, h=2, item_bits=8, mu=0)
    server = W.server_items(60, 8, seed)
    cfg.mu = P.server_bin_bound(60, 64)
    client = W.client_items(20, server, 9, 8, seed + 100)
    values = W.item_values(60, 1, 5000, seed + 500)
    ctx = Context.standard(cfg.n, cfg.L)
    sk, rlk = small_keys(ctx, seed + 200)
    ctab, cval, _, planes = PR.client_prepare(cfg, client)
    stab, sval, spos, _ = PR.server_prepare(cfg, server)
    vtab = PR.server_values(cfg, server, values)
    assert (vtab[sval == 0] == 0).all() and (vtab[sval == 1] > 0).all()
    cts = encrypt_planes(ctx, sk, planes, seed + 300)
    mask = W.zero_sum_mask(cfg.n, ctx.t, seed + 400)
    total = ctx.server_eval(cts, spos, rlk, cfg.h, mask=mask, vals=vtab)
    want = PR.plaintext_sum(client, server, values)
    assert want != 0
    assert PR.extract_sum(ctx.decrypt_slots(sk, total)) == want
    labels = ctx.decrypt_slots(sk, ctx.server_eval(cts, spos, rlk, cfg.h, vals=vtab))
    assert (labels == PR.plaintext_labels(ctab, cval, stab, sval, vtab)).all()
    assert np.count_nonzero(labels) == 9
    ones = np.ones_like(vtab)
    assert (ctx.server_eval(cts, spos, rlk, cfg.h, mask=mask, vals=ones) ==
            ctx.server_eval(cts, spos, rlk, cfg.h, mask=mask)).all()


@pytest.mark.slow
def test_toy_configuration_end_to_end():
    """N=4096, two primes, h=2, l=363, n=256 server / m=16 client 16-bit items, 4 planted."""
    cfg = PR.Config(n=4096, L=2, h=2, item_bits=16, mu=P.server_mu(256, 4096))
    ctx = Context.standard(cfg.n, cfg.L)
    server = W.server_items(256, 16, 11)
    client = W.client_items(16, server, 4, 16, 12)
    sk, rlk = small_keys(ctx, 13)
    _, _, _, planes = PR.client_prepare(cfg, client)
    _, _, spos, _ = PR.server_prepare(cfg, server)
    cts = encrypt_planes(ctx, sk, planes, 14)
    out = ctx.server_eval(cts, spos, rlk, cfg.h, mask=W.zero_sum_mask(cfg.n, ctx.t, 15))
    assert PR.extract_cardinality(ctx.decrypt_slots(sk, out)) == 4
    assert ctx.noise_budget(sk, out) > 0
