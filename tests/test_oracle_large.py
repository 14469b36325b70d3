"""Pins of the oracle's large-element path (Sec. 5 "Optimization for Large Elements", Lemma
"fail-collide"; Sec. 7 "Parameters for Large Elements"), on the CPU.

- lambda = alpha + ceil(log2(b mu_c mu_s)) reproduces the paper's own second form
  lambda_bar = lambda - log2(b) = 40 + ceil(log2 mu_s) for every row of Table "psisum-eval"
  (b = 16384), and its bound is at most 2^-alpha and more than 2^-(alpha + 1);
- the hash is SHA-256 (the FIPS 180-2 "abc" digest) truncated to lambda bits, nested in lambda;
- the Lemma, numerically: with tiny lambda the protocol's tables (cuckoo hashing of the client,
  simple hashing of the server, permutation-based hashing) on hashed disjoint sets report a match
  exactly when a client and a server element collide, and the observed failure rate stays below
  b mu_c mu_s 2^-lambda; with the paper's lambda none occurs;
- the whole protocol on hashed 32-byte elements (h = 16 over the stored bits, PSI-Sum with server
  values, and the cardinality): the decrypted results equal their plaintext definitions.
"""
import math

import numpy as np
import pytest

from oracle import hashing, large as LG, params as P, protocol as PR
from oracle.core import Context
import workload as W


def test_element_bits_match_the_paper(golden):
    rows = [r for r in golden["server_max_bin_load"]["rows"] if r[1] == 16384]
    assert [r[2] for r in rows] == [100, 296, 976, 3487]
    for n, b, mu in rows:
        lam = LG.element_bits(b, 1, mu)
        assert lam - int(math.log2(b)) == 40 + math.ceil(math.log2(mu))      # the paper's lambda_bar
        bound = LG.failure_bound(b, 1, mu, lam)
        assert bound <= 2 ** -40 < 2 * bound
    assert LG.element_bits(16384, 1, 296) == 63
    assert LG.ceil_log2(1) == 0 and LG.ceil_log2(2) == 1 and LG.ceil_log2(3) == 2 and LG.ceil_log2(1 << 20) == 20


def test_hash_is_truncated_sha256():
    digest = 0xba7816bf8f01cfea414140de5dae2223b00361a396177a9cb410ff61f20015ad   # SHA-256("abc")
    assert LG.hash_to_bits(b"abc", 64) == digest >> 192
    for lam in (1, 13, 40, 63):
        assert LG.hash_to_bits(b"abc", lam) == digest >> (256 - lam)
        assert LG.hash_to_bits(b"abc", 64) >> (64 - lam) == LG.hash_to_bits(b"abc", lam)
    vals = LG.hash_elements([bytes([i]) for i in range(200)], 20)
    assert vals.dtype == np.uint64 and int(vals.max()) < (1 << 20) and len(set(vals.tolist())) > 190


@pytest.mark.slow
def test_failure_rate_below_the_lemma():
    b, lam, mu, m, n, trials = 8, 10, 40, 3, 30, 3000
    fails = 0
    lam40 = LG.element_bits(b, 1, mu)
    for t in range(trials):
        # a client set whose cuckoo insertion fails (a separate protocol failure, reported as an
        # error) is drawn again: that depends on the client values only, not on their collisions
        # with the independent server values
        for retry in range(100):
            client = LG.random_elements(m, 8, 1000 + t + 10**6 * retry)
            hc = LG.hash_elements(client, lam)
            try:
                hashing.cuckoo_table(hc.tolist(), b, 0x5EED, 3, pbh_bits=lam)
                hashing.cuckoo_table(LG.hash_elements(client, lam40).tolist(), b, 0x5EED, 3, pbh_bits=lam40)
                break
            except (hashing.CuckooFailure, ValueError):
                continue
        server = LG.random_elements(n, 8, 900000 + t, exclude=client)
        hs = LG.hash_elements(server, lam)
        found = LG.table_matches(hc, hs, b, lam, mu)
        collide = len(set(hc.tolist()) & set(hs.tolist()))
        assert found == collide                       # a match is exactly a client-server collision
        fails += found > 0
        if t < 20:                                    # the paper's lambda on the same sets: no match
            assert LG.table_matches(LG.hash_elements(client, lam40), LG.hash_elements(server, lam40), b, lam40,
                                    mu) == 0
    rate = fails / trials
    bound = float(LG.failure_bound(b, 1, mu, lam))    # 8 * 40 / 1024
    union = 1 - (1 - 2.0 ** -lam) ** (m * n)          # any of the m n pairs colliding
    assert rate <= bound
    assert abs(rate - union) < 5 * math.sqrt(union * (1 - union) / trials)


@pytest.mark.slow
@pytest.mark.parametrize("with_values", [False, True])
def test_protocol_on_hashed_elements(with_values):
    log_n, L, h, n_server, m, planted = 10, 5, 16, 200, 24, 7
    n = 1 << log_n
    mu = P.server_bin_bound(n_server, n)
    lam = LG.element_bits(n, 1, mu)
    cfg = PR.Config(n=n, L=L, h=h, item_bits=lam, mu=mu, pbh=True)
    assert cfg.effective_bits == lam - log_n + 2 and cfg.ell == P.code_length(cfg.effective_bits, h)
    server_e = LG.random_elements(n_server, 32, 5)
    client_e = server_e[:planted] + LG.random_elements(m - planted, 32, 6, exclude=server_e)
    hs, hc = LG.hash_elements(server_e, lam), LG.hash_elements(client_e, lam)
    ctx = Context(n, P.select_primes(n, L))
    _, _, _, planes = PR.client_prepare(cfg, hc)
    _, _, spos, _ = PR.server_prepare(cfg, hs)
    sk = W.secret_key(n, 7)
    rlk = ctx.keygen_relin(sk, W.uniform_residues((L,), ctx.primes, n, 8, "rlk-a"), W.errors((L, n), 8, "rlk-e"))
    cts = PR.encrypt_planes(ctx, sk, planes, W.uniform_residues((cfg.ell,), ctx.primes, n, 9, "enc-a"),
                            W.errors((cfg.ell, n), 9, "enc-e"))
    mask = W.zero_sum_mask(n, ctx.t, 10)
    vals = None
    values = W.item_values(n_server, 1, 1 << 12, 11)
    if with_values:
        vals = PR.server_values(cfg, hs, values)
    out = ctx.server_eval(cts, spos, rlk, h, mask=mask, vals=vals)
    assert ctx.noise_budget(sk, out) > 0
    slots = ctx.decrypt_slots(sk, out)
    if with_values:
        assert PR.extract_sum(slots) == int(values[:planted].astype(np.int64).sum() % ctx.t)
    else:
        assert PR.extract_cardinality(slots) == planted
