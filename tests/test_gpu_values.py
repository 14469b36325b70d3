"""GPU parity of PSI-Sum (Alg. 5) and labelled PSI (Alg. 4): the server computation with server
values, against the oracle bit for bit, and batched / served / sampled full-size cases."""
import time

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


def setup_case(log_n, L, h, item_bits, n_server, m_client, planted, seed, cache, mu=None):
    import paper_2310_14565_amd as pk
    n = 1 << log_n
    mu = mu or P.server_bin_bound(n_server, n)
    cfg = PR.Config(n=n, L=L, h=h, item_bits=item_bits, mu=mu)
    gp = pk.Params(log_n, L, h, item_bits, mu, hash_seed=cfg.hash_seed)
    ctx = Context(n, gp.q_primes)
    server = W.server_items(n_server, item_bits, seed)
    client = W.client_items(m_client, server, planted, item_bits, seed + 1)
    values = W.item_values(n_server, 1, 60000, seed + 2)
    ctab, cval, _, planes = PR.client_prepare(cfg, client)
    stab, sval, spos, _ = PR.server_prepare(cfg, server)
    vtab = PR.server_values(cfg, server, values)
    sk = W.secret_key(n, seed + 3)
    rlk = ctx.keygen_relin(sk, W.uniform_residues((L,), ctx.primes, n, seed + 4, "rlk-a"),
                           W.errors((L, n), seed + 4, "rlk-e"))
    cts = PR.encrypt_planes(ctx, sk, planes, W.uniform_residues((cfg.ell,), ctx.primes, n, seed + 5, "enc-a"),
                            W.errors((cfg.ell, n), seed + 5, "enc-e"))
    sv = pk.Server(gp, server, cache_plaintexts=cache, values=values)
    say(f"values log_n={log_n} L={L} h={h} ell={cfg.ell} mu={mu} max_load={sv.max_load} cache={cache}")
    return dict(gp=gp, ctx=ctx, cfg=cfg, server=server, client=client, values=values, ctab=ctab, cval=cval,
                stab=stab, sval=sval, spos=spos, vtab=vtab, sk=sk, rlk=rlk, cts=cts, sv=sv)


@pytest.mark.parametrize("h,item_bits,cache", [(1, 9, False), (2, 10, True), (3, 12, False), (4, 12, True)])
def test_psi_sum_and_labels_match_oracle(h, item_bits, cache):
    c = setup_case(10, 3, h, item_bits, n_server=200, m_client=40, planted=9, seed=60 + h, cache=cache)
    ctx, sk, gp = c["ctx"], c["sk"], c["gp"]
    L, n = gp.L, gp.n
    d_cts, d_rlk = to_dev(c["cts"]), to_dev(c["rlk"])
    mask = W.zero_sum_mask(n, ctx.t, 70 + h)
    # PSI-Sum
    out = empty((2, L, n), np.uint64)
    c["sv"].eval(d_cts, d_rlk, to_dev(mask), out)
    got = to_host(out, np.uint64)
    want = ctx.server_eval(c["cts"], c["spos"], c["rlk"], h, mask=mask, vals=c["vtab"])
    assert (got == want).all()
    assert PR.extract_sum(ctx.decrypt_slots(sk, got)) == PR.plaintext_sum(c["client"], c["server"], c["values"])
    assert ctx.noise_budget(sk, got) > 0
    # labelled PSI
    c["sv"].eval(d_cts, d_rlk, None, out)
    got = to_host(out, np.uint64)
    assert (got == ctx.server_eval(c["cts"], c["spos"], c["rlk"], h, vals=c["vtab"])).all()
    labels = ctx.decrypt_slots(sk, got)
    assert (labels == PR.plaintext_labels(c["ctab"], c["cval"], c["stab"], c["sval"], c["vtab"])).all()
    assert np.count_nonzero(labels) == 9
    # a range without finalisation
    sv = c["sv"]
    sv.eval_range(d_cts, d_rlk, 1, 3, False, None, out)
    assert (to_host(out, np.uint64) ==
            ctx.server_eval(c["cts"], c["spos"], c["rlk"], h, finalize=False, begin=1, end=3, vals=c["vtab"])).all()


def test_values_batched_and_served_equal_alone():
    import paper_2310_14565_amd as pk
    c = setup_case(10, 3, 4, 14, n_server=5000, m_client=60, planted=11, seed=80, cache=True)
    gp, ctx, sv = c["gp"], c["ctx"], c["sv"]
    L, n = gp.L, gp.n
    d_cts, d_rlk = to_dev(c["cts"]), to_dev(c["rlk"])
    masks = [to_dev(W.zero_sum_mask(n, ctx.t, 90 + i)) if i % 2 == 0 else None for i in range(5)]
    alone = []
    for m in masks:
        o = empty((2, L, n), np.uint64)
        sv.eval(d_cts, d_rlk, m, o)
        alone.append(to_host(o, np.uint64).copy())
    outs = [empty((2, L, n), np.uint64) for _ in masks]
    sv.eval_batch([d_cts] * len(masks), [d_rlk] * len(masks), masks, outs)
    for i, o in enumerate(outs):
        assert (to_host(o, np.uint64) == alone[i]).all(), f"batched {i}"
    srv = pk.Serve(sv, max_active=2)
    souts = [empty((2, L, n), np.uint64) for _ in masks]
    ids = [srv.submit(d_cts, d_rlk, m, o) for m, o in zip(masks[:2], souts[:2])]
    time.sleep(0.02)
    ids += [srv.submit(d_cts, d_rlk, m, o) for m, o in zip(masks[2:], souts[2:])]
    for r in ids:
        srv.wait(r)
    srv.close()
    for i, o in enumerate(souts):
        assert (to_host(o, np.uint64) == alone[i]).all(), f"served {i}"
    assert PR.extract_sum(ctx.decrypt_slots(c["sk"], alone[0])) == \
        PR.plaintext_sum(c["client"], c["server"], c["values"])


def test_value_range_checked():
    import paper_2310_14565_amd as pk
    gp = pk.Params(10, 3, 2, 10, P.server_bin_bound(100, 1024))
    items = W.server_items(100, 10, 5)
    vals = np.zeros(100, np.uint32)
    vals[7] = 65537
    with pytest.raises(pk.PepsiError):
        pk.Server(gp, items, values=vals)


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_psi_sum_paper_size_sampled():
    """Paper-shaped PSI-Sum (n = 2^20, N = 8192, h = 4), cached plaintexts: sampled batches
    against the oracle, and an encrypted query's decrypted sum."""
    import torch
    import bench
    import paper_2310_14565_amd as pk
    n, L, h, mu = 8192, 4, 4, 526
    gp = pk.Params(13, L, h, 32, mu)
    ctx = Context(n, gp.q_primes)
    cfg = PR.Config(n=n, L=L, h=h, item_bits=32, mu=mu)
    items = W.server_items(1 << 20, 32, 41)
    values = W.item_values(1 << 20, 0, 1 << 12, 42)
    sv = pk.Server(gp, items, cache_plaintexts=True, values=values)
    _, _, spos, _ = PR.server_prepare(cfg, items)
    vtab = PR.server_values(cfg, items, values)
    cts = W.uniform_residues((gp.ell, 2), ctx.primes, n, 43, "vals-cts")
    rlk = W.uniform_residues((L, 2), ctx.primes, n, 44, "vals-rlk")
    out = empty((2, L, n), np.uint64)
    for b in (5, sv.max_load - 1):
        sv.eval_range(to_dev(cts), to_dev(rlk), b, b + 1, False, None, out)
        want = ctx.server_eval(cts, spos, rlk, h, finalize=False, begin=b, end=b + 1, vals=vtab)
        assert (to_host(out, np.uint64) == want).all(), f"batch {b}"
    q = bench.make_query(gp, items, {"item_bits": 32}, 1024, 256, 46)
    client = q["client"]
    res = torch.zeros((2, L, n), dtype=torch.int64, device="cuda")
    sv.eval(q["cts"], q["rlk"], q["mask"], res)
    slots = torch.zeros((1, n), dtype=torch.int32, device="cuda")
    gp.decrypt(q["sk"], res.reshape(1, 2, L, n), slots)
    total = int(to_host(slots, np.uint32).astype(np.int64).sum() % 65537)
    assert total == PR.plaintext_sum(client, items, values)
    sv.close()
