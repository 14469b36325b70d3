"""Serving with continuous batching: requests admitted while others run; each result equals
its single-query result bit for bit."""
import time

import numpy as np
import pytest

from gpu_util import empty, say, to_dev, to_host
from oracle import params as P, protocol as PR
from oracle.core import Context
from test_gpu_batch import make_queries

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("h,cache", [(2, True), (4, False)])
def test_serving_mix_equals_alone(h, cache):
    import torch
    import paper_2310_14565_amd as pk
    import workload as W
    log_n, L, bits = 10, 3, 14
    n = 1 << log_n
    n_server = 6000                       # max load ~ 30 batches: several 16-batch tiles per cycle
    mu = P.server_bin_bound(n_server, n)
    cfg = PR.Config(n=n, L=L, h=h, item_bits=bits, mu=mu)
    gp = pk.Params(log_n, L, h, bits, mu, hash_seed=cfg.hash_seed)
    ctx = Context(n, gp.q_primes)
    server = W.server_items(n_server, bits, 90 + h)
    sv = pk.Server(gp, server, cache_plaintexts=cache)
    qs = make_queries(ctx, cfg, server, 11, 500 + h)
    say(f"serve h={h} max_load={sv.max_load} queries={len(qs)} planes={sv.plane_groups}")
    assert (sv.plane_groups > 0) == cache          # cached groups take the matrix-core path
    dev = [dict(cts=to_dev(q["cts"]), rlk=to_dev(q["rlk"]), mask=None if q["mask"] is None else to_dev(q["mask"]),
                out=empty((2, L, n), np.uint64)) for q in qs]
    alone = []
    for d in dev:
        o = empty((2, L, n), np.uint64)
        sv.eval(d["cts"], d["rlk"], d["mask"], o)
        alone.append(to_host(o, np.uint64))
    torch.cuda.synchronize()
    srv = pk.Serve(sv, max_active=4)
    assert srv.info().slots == 4
    ids = [srv.submit(d["cts"], d["rlk"], d["mask"], d["out"]) for d in dev[:6]]
    time.sleep(0.05)                       # the first requests are running
    ids += [srv.submit(d["cts"], d["rlk"], d["mask"], d["out"]) for d in dev[6:]]
    stats = [srv.wait(i) for i in ids]
    info = srv.info()
    srv.close()
    assert info.completed == len(qs) and info.active == 0 and info.queued == 0
    for i, d in enumerate(dev):
        assert (to_host(d["out"], np.uint64) == alone[i]).all(), f"request {i}"
        q = qs[i]
        if q["mask"] is not None:
            assert PR.extract_cardinality(ctx.decrypt_slots(q["sk"], alone[i])) == q["planted"]
    # more requests than slots: some waited in the queue, and some were admitted while others ran
    admits = sorted(s.admit_s for s in stats)
    dones = sorted(s.done_s for s in stats)
    assert admits[-1] > dones[0]
    assert all(s.done and s.done_s >= s.admit_s >= s.submit_s for s in stats)


def test_serving_budget_too_small():
    import paper_2310_14565_amd as pk
    import workload as W
    gp = pk.Params(10, 3, 2, 10, P.server_bin_bound(300, 1024))
    sv = pk.Server(gp, W.server_items(300, 10, 5))
    with pytest.raises(pk.PepsiError):
        pk.Serve(sv, max_active=4, hbm_budget=1 << 20)


def test_serving_admission_by_memory():
    """A budget of k slots' device bytes gives exactly k slots: k requests run at once, the rest
    wait in the queue (no failure), and every result equals its single-query result."""
    import torch
    import paper_2310_14565_amd as pk
    import workload as W
    log_n, L, h, bits, n_server = 10, 3, 2, 14, 6000
    n = 1 << log_n
    mu = P.server_bin_bound(n_server, n)
    cfg = PR.Config(n=n, L=L, h=h, item_bits=bits, mu=mu)
    gp = pk.Params(log_n, L, h, bits, mu, hash_seed=cfg.hash_seed)
    ctx = Context(n, gp.q_primes)
    server = W.server_items(n_server, bits, 191)
    sv = pk.Server(gp, server, cache_plaintexts=True)
    qs = make_queries(ctx, cfg, server, 7, 707)
    dev = [dict(cts=to_dev(q["cts"]), rlk=to_dev(q["rlk"]), mask=None if q["mask"] is None else to_dev(q["mask"]),
                out=empty((2, L, n), np.uint64)) for q in qs]
    alone = []
    for d in dev:
        o = empty((2, L, n), np.uint64)
        sv.eval(d["cts"], d["rlk"], d["mask"], o)
        alone.append(to_host(o, np.uint64))
    probe = pk.Serve(sv, max_active=1)
    per_slot = probe.info().slot_bytes
    probe.close()
    assert per_slot > 0
    k = 3
    srv = pk.Serve(sv, max_active=0, hbm_budget=k * per_slot + per_slot // 2)
    assert srv.info().slots == k
    ids = [srv.submit(d["cts"], d["rlk"], d["mask"], d["out"]) for d in dev]
    queued_seen = srv.info().queued
    stats = [srv.wait(i) for i in ids]
    info = srv.info()
    srv.close()
    say(f"admission by memory: {per_slot} bytes per slot, {info.slots} slots, {queued_seen} queued at first")
    assert info.completed == len(dev) and info.queued == 0
    assert queued_seen >= 1                             # requests beyond the slots waited in the queue
    assert {s.slot for s in stats} == set(range(k))     # every slot used, none beyond the budget
    admits = sorted(s.admit_s for s in stats)
    assert admits[k] > admits[k - 1]                    # the (k+1)-th request waited for a slot
    for i, d in enumerate(dev):
        assert (to_host(d["out"], np.uint64) == alone[i]).all(), f"request {i}"

