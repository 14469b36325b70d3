"""Schedules of the batched evaluation: the launch sequence captured into a HIP graph and replayed,
eager launches, tile sizes and the select-and-sum kernel all give each query's single-query result
bit for bit.  Graph replays are checked one by one, with other work of the program (eager
evaluations, torch kernels, synchronisations, a second capture) between them."""
import numpy as np
import pytest

from gpu_util import empty, say, to_dev, to_host
from oracle import params as P, protocol as PR
from oracle.core import Context
from test_gpu_batch import make_queries
import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def setup():
    import paper_2310_14565_amd as pk
    log_n, L, h, bits, n_server = 10, 3, 4, 16, 12000
    n = 1 << log_n
    mu = P.server_bin_bound(n_server, n)
    cfg = PR.Config(n=n, L=L, h=h, item_bits=bits, mu=mu)
    gp = pk.Params(log_n, L, h, bits, mu, hash_seed=cfg.hash_seed)
    ctx = Context(n, gp.q_primes)
    server = W.server_items(n_server, bits, 123)
    sv = pk.Server(gp, server, cache_plaintexts=True)
    assert sv.plane_groups > 0
    qs = make_queries(ctx, cfg, server, 6, 31337)
    d = [dict(cts=to_dev(q["cts"]), rlk=to_dev(q["rlk"]), mask=None if q["mask"] is None else to_dev(q["mask"]))
         for q in qs]
    alone = []
    for x in d:
        o = empty((2, L, n), np.uint64)
        sv.eval(x["cts"], x["rlk"], x["mask"], o)
        alone.append(to_host(o, np.uint64).copy())
    _, _, spos, _ = PR.server_prepare(cfg, server)
    want0 = ctx.server_eval(qs[0]["cts"], spos, qs[0]["rlk"], h, mask=qs[0]["mask"])
    assert (alone[0] == want0).all()
    yield dict(pk=pk, sv=sv, d=d, alone=alone, L=L, n=n)
    sv.close()


def _batch(st, outs, idx):
    d = st["d"]
    st["sv"].eval_batch([d[i]["cts"] for i in idx], [d[i]["rlk"] for i in idx], [d[i]["mask"] for i in idx], outs)


def _check(st, outs, idx, what):
    for o, i in zip(outs, idx):
        assert (to_host(o, np.uint64) == st["alone"][i]).all(), f"{what}: query {i}"


def test_graph_replays(setup):
    import torch
    st, pk = setup, setup["pk"]
    sv = st["sv"]
    sv.set_schedule(graph=pk.GRAPH_ON)
    sch = sv.schedule(4).as_dict()
    say(f"schedule for 4 queries: {sch}")
    assert sch["graph"] == "captured HIP graph"
    idx = [0, 1, 2, 3]
    outs = [empty((2, st["L"], st["n"]), np.uint64) for _ in idx]
    for rep in range(4):
        for o in outs:
            o.fill_(7)                                      # eager torch work between replays
        _batch(st, outs, idx)                               # rep 0 captures, later reps replay
        if rep == 2:                                        # eager evaluation of the same server
            o = empty((2, st["L"], st["n"]), np.uint64)
            sv.eval(st["d"][4]["cts"], st["d"][4]["rlk"], st["d"][4]["mask"], o)
            assert (to_host(o, np.uint64) == st["alone"][4]).all()
        torch.cuda.synchronize()
        _check(st, outs, idx, f"replay {rep}")
    # other buffers: a second graph; then the first one again
    idx2 = [5, 4, 3, 2]
    outs2 = [empty((2, st["L"], st["n"]), np.uint64) for _ in idx2]
    _batch(st, outs2, idx2)
    _check(st, outs2, idx2, "second graph")
    for o in outs:
        o.zero_()
    _batch(st, outs, idx)
    _check(st, outs, idx, "first graph again")
    sv.set_schedule(reset=True)


@pytest.mark.parametrize("tile,kernel,graph,run", [(16, 1, 2, 2), (32, 1, 1, 2), (64, 1, 2, 2), (16, 2, 1, 2),
                                                   (64, 2, 2, 2), (16, 1, 1, 1), (32, 1, 2, 1), (64, 1, 1, 1)])
def test_schedules_equal_alone(setup, tile, kernel, graph, run):
    """run = 1: the select-and-sum of a run of tiles in one launch (request planes staged once per
    run), the tiles' product trees after it."""
    st = setup
    sv = st["sv"]
    sv.set_schedule(tile_batches=tile, select_kernel=kernel, graph=graph, run=run)
    sch = sv.schedule(6)
    assert (sch.tile_batches, sch.select_kernel, sch.graph, sch.run, sch.source) == (tile, kernel, graph, run, 2)
    idx = [0, 1, 2, 3, 4, 5]
    outs = [empty((2, st["L"], st["n"]), np.uint64) for _ in idx]
    for rep in range(2):
        _batch(st, outs, idx)
        _check(st, outs, idx, f"tile {tile} kernel {kernel} graph {graph} run {run} rep {rep}")
    sv.set_schedule(reset=True)


def test_schedule_arguments(setup):
    pk = setup["pk"]
    sv = setup["sv"]
    for bad in (dict(tile_batches=8), dict(select_kernel=3), dict(graph=5), dict(run=3)):
        with pytest.raises(pk.PepsiError):
            sv.set_schedule(**bad)
    sv.set_schedule(reset=True)
    assert sv.schedule(3).source in (0, 1)


def test_event_timing_counts(setup):
    """pepsi_server_timing: a plain evaluation's select-and-sum, transforms, rescales and
    extensions are timed, with the product counts the header states (h = 4: two first-level
    products per pair sharing their squares, one second-level product, the last level's
    relinearisation deferred)."""
    st = setup
    sv, L, n = st["sv"], st["L"], st["n"]
    K = L + 1
    x = st["d"][0]
    o = empty((2, L, n), np.uint64)
    sv.timing(enable=True, reset=True)
    sv.eval(x["cts"], x["rlk"], x["mask"], o)
    tm = sv.timing(enable=False)
    assert (to_host(o, np.uint64) == st["alone"][0]).all()
    assert tm.evals == 1 and tm.eval_ms > 0
    assert tm.select_sum_launches >= 1 and tm.select_sum_ms > 0
    assert tm.ntt_fwd_rows > 0 and tm.ntt_inv_rows > 0
    npairs = sv.max_load                       # batches at or above the fullest bin are skipped
    base = (L + K) + K * (L + 1) + K + L * (K + 1)
    j0 = 2
    assert tm.rescale_products == npairs * n * ((2 * j0 + 1) * base + 2 * j0 * (L + K) + 3 * base)
    assert tm.ext_products == npairs * n * (L + K * (L + 1)) * (2 + 2 * j0)
    assert tm.rescale_launches >= 2 and tm.rescale_ms > 0 and tm.ext_launches >= 2 and tm.ext_ms > 0
