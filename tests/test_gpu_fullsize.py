"""Parity at the full workload sizes, in the configuration the benchmark times.

The oracle evaluates sampled server batches one by one (a full query takes it tens of minutes
at N = 8192 and hours at N = 16384); the GPU evaluates the same batches alone, and the whole
range in its normal tiles, which must equal the sum of per-chunk ranges (sums mod Q are exact,
so tiling cannot change a bit).  A real encrypted query of each size must decrypt to its
planted cardinality.  Request ciphertexts of the sampled comparisons are seeded uniform
residues: the server computation is defined on any ciphertext.
"""
import numpy as np
import pytest

from gpu_util import empty, to_dev, to_host
from oracle import protocol as PR
from oracle.core import Context

pytestmark = pytest.mark.gpu

CASES = {
    # Paper-shaped query (n = 2^20, m = 1024), plaintexts resident as in the benchmark.
    # The range starts inside a 16-batch group of the plaintext store and its launch spans three
    # batch groups of the select-and-sum, the last one partial.
    "paper": dict(log_n=13, L=4, h=4, bits=32, mu=526, n=1 << 20, m=1024, planted=256, cache=True,
                  samples=(0, 233, -1), ranges=((216, 249),), chunk=50),
    # Large configuration (N = 16384, 8 primes, n = 2^24, m = 4096): plaintexts generated per tile.
    "large": dict(log_n=14, L=8, h=4, bits=32, mu=3487, n=1 << 24, m=4096, planted=1024, cache=False,
                  samples=(-1,), ranges=(), chunk=800),
}


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _progress(capsys, msg):
    with capsys.disabled():
        print(f"    [{msg}]", flush=True)


def _add(a, b, primes):
    q = np.array(primes, dtype=np.uint64)[None, :, None]
    return (a + b) % q


@pytest.mark.slow
@pytest.mark.timeout(1000)
@pytest.mark.parametrize("name", ["paper", "large"])
def test_full_size(name, capsys):
    import torch
    import bench
    import paper_2310_14565_amd as pk
    import workload as W
    c = CASES[name]
    n, L = 1 << c["log_n"], c["L"]
    gp = pk.Params(c["log_n"], L, c["h"], c["bits"], c["mu"])
    ctx = Context(n, gp.q_primes)
    cfg = PR.Config(n=n, L=L, h=c["h"], item_bits=c["bits"], mu=c["mu"])
    items = W.server_items(c["n"], c["bits"], 31)
    _progress(capsys, f"{name}: server set of {c['n']} items, GPU preparation")
    sv = pk.Server(gp, items, cache_plaintexts=c["cache"])
    _progress(capsys, f"{name}: max load {sv.max_load}, cached batches {sv.cached_batches}; oracle tables")
    _, _, spos, _ = PR.server_prepare(cfg, items)
    assert (sv.codewords() == spos).all()                  # hashing and CW encoding, bit-exact

    # sampled batches against the oracle
    cts = W.uniform_residues((gp.ell, 2), ctx.primes, n, 32, "full-cts")
    rlk = W.uniform_residues((L, 2), ctx.primes, n, 33, "full-rlk")
    d_cts, d_rlk = to_dev(cts), to_dev(rlk)
    out = empty((2, L, n), np.uint64)
    for b in c["samples"]:
        b = b % sv.max_load
        sv.eval_range(d_cts, d_rlk, b, b + 1, False, None, out)
        got = to_host(out, np.uint64).copy()
        _progress(capsys, f"{name}: oracle batch {b}")
        want = ctx.server_eval(cts, spos, rlk, c["h"], finalize=False, begin=b, end=b + 1)
        assert (got == want).all(), f"batch {b}"
    for b0, b1 in c["ranges"]:
        sv.eval_range(d_cts, d_rlk, b0, b1, False, None, out)
        got = to_host(out, np.uint64).copy()
        _progress(capsys, f"{name}: oracle batches [{b0}, {b1})")
        want = ctx.server_eval(cts, spos, rlk, c["h"], finalize=False, begin=b0, end=b1)
        assert (got == want).all(), f"batches [{b0}, {b1})"

    # the whole range in the normal tiles equals the sum of chunked ranges
    _progress(capsys, f"{name}: whole range vs chunks")
    sv.eval_range(d_cts, d_rlk, 0, sv.max_load, False, None, out)
    whole = to_host(out, np.uint64).copy()
    total = np.zeros_like(whole)
    for b0 in range(0, sv.max_load, c["chunk"]):
        sv.eval_range(d_cts, d_rlk, b0, min(sv.max_load, b0 + c["chunk"]), False, None, out)
        total = _add(total, to_host(out, np.uint64), ctx.primes)
    assert (whole == total).all()
    del d_cts, d_rlk

    # a real encrypted query: cardinality and noise budget
    _progress(capsys, f"{name}: encrypted query")
    q = bench.make_query(gp, items, {"item_bits": c["bits"]}, c["m"], c["planted"], 34)
    res = torch.zeros((2, L, n), dtype=torch.int64, device="cuda")
    sv.eval(q["cts"], q["rlk"], q["mask"], res)
    slots = torch.zeros((1, n), dtype=torch.int32, device="cuda")
    gp.decrypt(q["sk"], res.reshape(1, 2, L, n), slots)
    card = int(to_host(slots, np.uint32).astype(np.int64).sum() % 65537)
    budget = gp.noise_budget(q["sk"], res)
    _progress(capsys, f"{name}: cardinality {card}, noise budget {budget} bits")
    assert card == c["planted"] and budget > 0

    # the batched path at full size: each query's result equals its single-query result
    q2 = bench.make_query(gp, items, {"item_bits": c["bits"]}, c["m"] // 2, c["planted"] // 2, 35)
    alone2 = torch.zeros_like(res)
    sv.eval(q2["cts"], q2["rlk"], q2["mask"], alone2)
    qs = [q, q2, q]
    outs = [torch.zeros_like(res) for _ in qs]
    if c["cache"]:
        # digit planes of every cached group, tiles of up to 64 batches on the matrix cores
        assert sv.plane_groups == -(-sv.cached_batches // 16) > 0
    else:
        # plaintexts generated per 16-batch tile, shared by the queries of the batch
        assert sv.plane_groups == 0 and sv.cached_batches == 0
    _progress(capsys, f"{name}: batched path, {len(qs)} queries")
    sv.eval_batch([x["cts"] for x in qs], [x["rlk"] for x in qs], [x["mask"] for x in qs], outs)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], res) and torch.equal(outs[2], res) and torch.equal(outs[1], alone2)
    if c["cache"]:
        # the select-and-sum of all batches in one matrix-core launch (request planes staged once)
        sv.set_schedule(run=pk.RUN_ON)
        assert sv.schedule(3).run == pk.RUN_ON
        for o in outs:
            o.zero_()
        _progress(capsys, f"{name}: batched path in one select-and-sum run")
        sv.eval_batch([x["cts"] for x in qs], [x["rlk"] for x in qs], [x["mask"] for x in qs], outs)
        torch.cuda.synchronize()
        assert torch.equal(outs[0], res) and torch.equal(outs[2], res) and torch.equal(outs[1], alone2)
        sv.set_schedule(reset=True)
    sv.close()

