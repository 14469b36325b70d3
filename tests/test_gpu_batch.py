"""Batched server computation: each query's result equals its result alone, bit for bit."""
import numpy as np
import pytest

from gpu_util import empty, say, to_dev, to_host
from oracle import params as P, protocol as PR
from oracle.core import Context
import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def make_queries(ctx, cfg, server, nq, seed):
    out = []
    for q in range(nq):
        m = int(W.rng(seed + q, "m").integers(8, 60))
        planted = m // 4
        client = W.client_items(m, server, planted, cfg.item_bits, seed + 17 * q)
        _, _, _, planes = PR.client_prepare(cfg, client)
        sk = W.secret_key(ctx.n, seed + 1000 + q)
        rlk = ctx.keygen_relin(sk, W.uniform_residues((ctx.L,), ctx.primes, ctx.n, seed + 2000 + q, "rlk-a"),
                               W.errors((ctx.L, ctx.n), seed + 2000 + q, "rlk-e"))
        cts = PR.encrypt_planes(ctx, sk, planes,
                                W.uniform_residues((cfg.ell,), ctx.primes, ctx.n, seed + 3000 + q, "enc-a"),
                                W.errors((cfg.ell, ctx.n), seed + 3000 + q, "enc-e"))
        mask = W.zero_sum_mask(ctx.n, ctx.t, seed + 4000 + q) if q % 3 != 2 else None
        out.append(dict(sk=sk, rlk=rlk, cts=cts, mask=mask, planted=planted))
    return out


@pytest.mark.parametrize("h,nq,cache,n_server", [(2, 1, False, 400), (2, 3, True, 400), (4, 9, True, 400),
                                                 (3, 17, False, 400), (2, 5, True, 12000), (4, 3, False, 12000),
                                                 (3, 70, True, 12000)])
def test_batch_equals_alone(h, nq, cache, n_server):
    """Small sets give tiles of a few batches; 12000 items give full 16-batch groups (one 54-batch
    tile with digit planes for up to 64 queries, 16-batch tiles beyond)."""
    import paper_2310_14565_amd as pk
    log_n, L = 10, 3
    bits = 16 if n_server > 1000 else {2: 10, 3: 12, 4: 12}[h]
    n = 1 << log_n
    mu = P.server_bin_bound(n_server, n)
    cfg = PR.Config(n=n, L=L, h=h, item_bits=bits, mu=mu)
    gp = pk.Params(log_n, L, h, bits, mu, hash_seed=cfg.hash_seed)
    ctx = Context(n, gp.q_primes)
    server = W.server_items(n_server, bits, 70 + h)
    sv = pk.Server(gp, server, cache_plaintexts=cache)
    qs = make_queries(ctx, cfg, server, nq, 100 * h + nq)
    say(f"batch h={h} nq={nq} cache={cache} ell={cfg.ell} max_load={sv.max_load} planes={sv.plane_groups}")
    if cache and sv.max_load >= 16:
        # whole 16-batch groups cached: the tiles take the matrix-core select-and-sum
        assert sv.plane_groups == -(-sv.cached_batches // 16) > 0
    d_cts = [to_dev(q["cts"]) for q in qs]
    d_rlk = [to_dev(q["rlk"]) for q in qs]
    d_mask = [None if q["mask"] is None else to_dev(q["mask"]) for q in qs]
    outs = [empty((2, L, n), np.uint64) for _ in qs]
    sv.eval_batch(d_cts, d_rlk, d_mask, outs)
    got = [to_host(o, np.uint64) for o in outs]
    for i, q in enumerate(qs):
        alone = empty((2, L, n), np.uint64)
        sv.eval(d_cts[i], d_rlk[i], d_mask[i], alone)
        assert (to_host(alone, np.uint64) == got[i]).all(), f"query {i}"
        slots = ctx.decrypt_slots(q["sk"], got[i])
        if q["mask"] is not None:
            assert PR.extract_cardinality(slots) == q["planted"]
    # one query against the oracle
    _, _, spos, _ = PR.server_prepare(cfg, server)
    want = ctx.server_eval(qs[-1]["cts"], spos, qs[-1]["rlk"], h, mask=qs[-1]["mask"])
    assert (got[-1] == want).all()


def test_code_length_beyond_planes_limit():
    """h = 1 over 13-bit items gives ell = 8192, beyond the 4096 positions for which the int8
    digit-plane contraction is exact: the server keeps no digit planes even when asked for them
    only, and the batched path runs on the 64-bit kernels with the same results."""
    import paper_2310_14565_amd as pk
    log_n, L, h, bits, n_server = 10, 2, 1, 13, 200
    n = 1 << log_n
    mu = P.server_bin_bound(n_server, n)
    cfg = PR.Config(n=n, L=L, h=h, item_bits=bits, mu=mu)
    gp = pk.Params(log_n, L, h, bits, mu, hash_seed=cfg.hash_seed)
    assert gp.ell == cfg.ell == 8192
    ctx = Context(n, gp.q_primes)
    server = W.server_items(n_server, bits, 77)
    sv = pk.Server(gp, server, cache_plaintexts=True, planes_only=True)
    assert sv.plane_groups == 0 and sv.cached_batches == sv.max_load
    qs = make_queries(ctx, cfg, server, 2, 8080)
    d_cts = [to_dev(q["cts"]) for q in qs]
    d_rlk = [to_dev(q["rlk"]) for q in qs]
    d_mask = [None if q["mask"] is None else to_dev(q["mask"]) for q in qs]
    outs = [empty((2, L, n), np.uint64) for _ in qs]
    sv.eval_batch(d_cts, d_rlk, d_mask, outs)
    _, _, spos, _ = PR.server_prepare(cfg, server)
    for i, q in enumerate(qs):
        got = to_host(outs[i], np.uint64)
        want = ctx.server_eval(q["cts"], spos, q["rlk"], h, mask=q["mask"])
        assert (got == want).all(), f"query {i}"
    sv.close()
