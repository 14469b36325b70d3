"""A bounded plaintext cache: tiles inside the cached batches read the cache, the rest are
generated per evaluation, and every result is the same bit for bit whatever the bound."""
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


LOG_N, L, H, BITS, N_SERVER = 10, 3, 3, 16, 12000     # max load ~ 40-50 batches: 3-4 tiles of 16


@pytest.fixture(scope="module")
def case():
    import paper_2310_14565_amd as pk
    n = 1 << LOG_N
    mu = P.server_bin_bound(N_SERVER, n)
    cfg = PR.Config(n=n, L=L, h=H, item_bits=BITS, mu=mu)
    gp = pk.Params(LOG_N, L, H, BITS, mu, hash_seed=cfg.hash_seed)
    ctx = Context(n, gp.q_primes)
    server = W.server_items(N_SERVER, BITS, 71)
    values = W.item_values(N_SERVER, 1, 60000, 72)
    qs = make_queries(ctx, cfg, server, 3, 910)
    dev = [dict(cts=to_dev(q["cts"]), rlk=to_dev(q["rlk"]),
                mask=None if q["mask"] is None else to_dev(q["mask"])) for q in qs]
    return dict(pk=pk, n=n, cfg=cfg, gp=gp, ctx=ctx, server=server, values=values, qs=qs, dev=dev)


def _results(c, sv):
    """eval of every query, eval_batch of all, and a sum of eval_range over ragged ranges."""
    n = c["n"]
    alone = []
    for d in c["dev"]:
        o = empty((2, L, n), np.uint64)
        sv.eval(d["cts"], d["rlk"], d["mask"], o)
        alone.append(to_host(o, np.uint64))
    outs = [empty((2, L, n), np.uint64) for _ in c["dev"]]
    sv.eval_batch([d["cts"] for d in c["dev"]], [d["rlk"] for d in c["dev"]], [d["mask"] for d in c["dev"]], outs)
    batch = [to_host(o, np.uint64) for o in outs]
    d = c["dev"][0]
    cuts = [0, 5, 16, 19, 37, sv.max_load]
    parts = []
    for b0, b1 in zip(cuts[:-1], cuts[1:]):
        if b0 >= b1:
            continue
        o = empty((2, L, n), np.uint64)
        sv.eval_range(d["cts"], d["rlk"], b0, b1, False, None, o)
        parts.append(to_host(o, np.uint64).astype(object))
    primes = np.array(c["gp"].q_primes, dtype=object)[None, :, None]
    ranged = (sum(parts) % primes).astype(np.uint64)
    return alone, batch, ranged


@pytest.mark.parametrize("valued", [False, True])
def test_results_do_not_depend_on_the_cache_bound(case, valued):
    c = case
    pk = c["pk"]
    vals = c["values"] if valued else None
    ref_sv = pk.Server(c["gp"], c["server"], cache_plaintexts=False, values=vals)
    assert ref_sv.max_load > 37, "the ranges and bounds assume more than two 16-batch tiles"
    ref = _results(c, ref_sv)
    say(f"cache bound valued={valued} max_load={ref_sv.max_load}: uncached reference done")
    ml = ref_sv.max_load
    for bound in (16, 20, 37, 0, 10 ** 6, 5):
        want_cached = min(bound, ml) if bound else ml
        if want_cached < ml:
            want_cached -= want_cached % 16          # whole 16-batch tiles unless every batch is kept
        sv = pk.Server(c["gp"], c["server"], cache_plaintexts=True, values=vals, max_cached=bound)
        assert sv.cached_batches == want_cached, bound
        assert sv.cached == (want_cached > 0)
        got = _results(c, sv)
        say(f"  bound {bound}: {sv.cached_batches} cached batches")
        for kind, a, b in zip(("eval", "eval_batch"), ref[:2], got[:2]):
            for i, (x, y) in enumerate(zip(a, b)):
                assert (x == y).all(), f"{kind} query {i} bound {bound}"
        assert (ref[2] == got[2]).all(), f"eval_range bound {bound}"
        sv.close()
    # the first query against the oracle
    _, _, spos, _ = PR.server_prepare(c["cfg"], c["server"])
    vtab = PR.server_values(c["cfg"], c["server"], vals) if valued else None
    q = c["qs"][0]
    want = c["ctx"].server_eval(q["cts"], spos, q["rlk"], H, mask=q["mask"], vals=vtab)
    assert (ref[0][0] == want).all() and (ref[1][0] == want).all()
    ref_sv.close()


@pytest.mark.parametrize("valued,bound", [(False, 0), (True, 0), (False, 37)])
def test_planes_only_equals_uncached(case, valued, bound):
    """Plaintexts kept only as digit planes (all groups, or the first two under a bound of 37):
    single, ranged (group-aligned and not), batched and served results equal the uncached
    server's bit for bit."""
    import torch
    c = case
    pk = c["pk"]
    vals = c["values"] if valued else None
    ref_sv = pk.Server(c["gp"], c["server"], cache_plaintexts=False, values=vals)
    ref = _results(c, ref_sv)
    sv = pk.Server(c["gp"], c["server"], cache_plaintexts=True, values=vals, max_cached=bound, planes_only=True)
    ml = ref_sv.max_load
    want_groups = -(-ml // 16) if bound == 0 else bound // 16
    say(f"planes only valued={valued} bound={bound}: {sv.plane_groups} groups, max_load={ml}")
    assert sv.plane_groups == want_groups and sv.cached_batches == 0 and not sv.cached
    got = _results(c, sv)
    for kind, a, b in zip(("eval", "eval_batch"), ref[:2], got[:2]):
        for i, (x, y) in enumerate(zip(a, b)):
            assert (x == y).all(), f"{kind} query {i}"
    assert (ref[2] == got[2]).all(), "eval_range"
    # served
    n = c["n"]
    srv = pk.Serve(sv, max_active=2)
    outs = [empty((2, L, n), np.uint64) for _ in c["dev"]]
    ids = [srv.submit(d["cts"], d["rlk"], d["mask"], o) for d, o in zip(c["dev"], outs)]
    for r in ids:
        srv.wait(r)
    srv.close()
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        assert (to_host(o, np.uint64) == ref[0][i]).all(), f"served query {i}"
    sv.close()
    ref_sv.close()
