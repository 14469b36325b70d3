"""Pins of permutation-based hashing (Sec. 3.3) in the oracle: the (bin, stored value) map is
invertible, so equal values in equal bins mean equal elements; tables hold every element the
right number of times; the encrypted protocol with PBH gives the plaintext answers; and the
paper's 32-bit parameters (b = 2^13, h = 8) give its l = 24 for lambda_bar = 19 and l = 27 once
the hash-function index is stored."""
import itertools

import numpy as np
import pytest

from oracle import hashing as H, params as P, protocol as PR
from oracle.core import Context
import workload as W
from test_oracle_server import encrypt_planes, small_keys


def _invert(b, v, i_bits_low, seed, n_bins):
    """Element from (bin, stored value): i from the value's top bits, x_L its low bits, and
    x_H = bin XOR H_i(x_L)."""
    i = (v >> i_bits_low) + 1
    xl = v & ((1 << i_bits_low) - 1)
    xh = b ^ H.bin_of(xl, i, seed, n_bins)
    return (xh << i_bits_low) | xl


def test_pbh_placement_is_injective_exhaustive():
    lam, c, seed = 12, 6, 77
    n_bins = 1 << c
    seen = set()
    for x, i in itertools.product(range(1 << lam), (1, 2, 3)):
        b, v = H.pbh_place(x, i, seed, n_bins, lam)
        assert 0 <= b < n_bins and v < 3 << (lam - c)
        assert (b, v) not in seen
        seen.add((b, v))
        assert _invert(b, v, lam - c, seed, n_bins) == x
    assert len(seen) == 3 << lam


def test_pbh_tables_hold_each_element():
    lam, n_bins, seed = 20, 1 << 10, 0x5EED
    server = W.server_items(2000, lam, 5)
    client = W.client_items(600, server, 150, lam, 6)
    tab, val = H.cuckoo_table(client, n_bins, seed, 3, 500, pbh_bits=lam)
    got = sorted(_invert(k, int(tab[k]), lam - 10, seed, n_bins) for k in range(n_bins) if val[k])
    assert got == sorted(int(x) for x in client)
    mu = P.server_bin_bound(2000, n_bins)
    st, sv, _, idx = H.simple_table(server, n_bins, mu, seed, 3, pbh_bits=lam, with_index=True)
    assert sv.sum() == 3 * len(server)                         # one entry per hash function
    for r, k in zip(*np.nonzero(sv)):
        assert _invert(k, int(st[r, k]), lam - 10, seed, n_bins) == int(server[idx[r, k]])
    # at most one server entry of a bin equals the client's value there, exactly for the common items
    common = set(client.tolist()) & set(server.tolist())
    hits = 0
    for k in range(n_bins):
        if val[k]:
            m = int(((st[:, k] == tab[k]) & (sv[:, k] == 1)).sum())
            assert m <= 1
            hits += m
    assert hits == len(common) == 150


def test_paper_32bit_parameters():
    cfg = PR.Config(n=8192, L=4, h=8, item_bits=32, mu=526, pbh=True)
    assert cfg.item_bits - 13 == 19 and P.code_length(19, 8) == 24   # the paper's lambda_bar, l
    assert cfg.effective_bits == 21 and cfg.ell == 27                # with the hash index stored


@pytest.mark.parametrize("seed", [7, 8])
def test_small_psi_with_pbh(seed):
    cfg = PR.Config(n=64, L=3, h=2, item_bits=12, mu=0, pbh=True)
    server = W.server_items(70, 12, seed)
    cfg.mu = P.server_bin_bound(70, 64)
    client = W.client_items(24, server, 10, 12, seed + 100)
    values = W.item_values(70, 1, 3000, seed + 500)
    ctx = Context.standard(cfg.n, cfg.L)
    sk, rlk = small_keys(ctx, seed + 200)
    ctab, cval, _, planes = PR.client_prepare(cfg, client)
    stab, sval, spos, _ = PR.server_prepare(cfg, server)
    cts = encrypt_planes(ctx, sk, planes, seed + 300)
    mask = W.zero_sum_mask(cfg.n, ctx.t, seed + 400)
    card = ctx.decrypt_slots(sk, ctx.server_eval(cts, spos, rlk, cfg.h, mask=mask))
    assert PR.extract_cardinality(card) == 10
    ind = ctx.decrypt_slots(sk, ctx.server_eval(cts, spos, rlk, cfg.h))
    assert (ind == PR.plaintext_membership(ctab, cval, stab, sval)).all()
    vtab = PR.server_values(cfg, server, values)
    total = ctx.decrypt_slots(sk, ctx.server_eval(cts, spos, rlk, cfg.h, mask=mask, vals=vtab))
    assert PR.extract_sum(total) == PR.plaintext_sum(client, server, values)
