"""Degenerate sets: an empty server set (no batch holds an item), an empty client set (every
client slot a dummy), a single item on each side, and empty batch ranges.  Each result is
compared bit for bit with the oracle and decrypted."""
import numpy as np
import pytest

from gpu_util import empty, say, to_dev, to_host
from oracle import protocol as PR
from test_gpu_server import run_case
import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("n_server,m_client,planted,cache,mask", [
    (0, 30, 0, False, True), (0, 30, 0, True, False), (200, 0, 0, True, True), (0, 0, 0, False, True),
    (1, 1, 1, True, True), (1, 1, 0, False, False)])
def test_degenerate_sets(n_server, m_client, planted, cache, mask):
    gp, ctx, sv, cts, rlk, spos, sk = run_case(10, 3, 2, 10, n_server, m_client, planted, seed=31 + n_server,
                                              cache=cache, mask=mask)
    if n_server == 0:
        assert sv.max_load == 0 and (spos == 0xFFFF).all()


def test_empty_server_batched_and_ranges():
    """No batches: eval_batch gives each query what eval gives, and an empty range is the
    encryption of zero with zero noise, (0, 0)."""
    gp, ctx, sv, cts, rlk, spos, sk = run_case(10, 3, 3, 12, 0, 20, 0, seed=41)
    n, L = gp.n, gp.L
    cfg = PR.Config(n=n, L=L, h=3, item_bits=12, mu=gp.mu)
    qs = []
    for q in range(3):
        client = W.client_items(10 + 7 * q, np.zeros(0, np.uint32), 0, 12, 43 + q)
        _, _, _, planes = PR.client_prepare(cfg, client)
        qk = W.secret_key(n, 50 + q)
        qs.append(dict(sk=qk, cts=PR.encrypt_planes(ctx, qk, planes,
                                                     W.uniform_residues((cfg.ell,), ctx.primes, n, 60 + q, "enc-a"),
                                                     W.errors((cfg.ell, n), 60 + q, "enc-e")),
                       rlk=ctx.keygen_relin(qk, W.uniform_residues((L,), ctx.primes, n, 70 + q, "rlk-a"),
                                            W.errors((L, n), 70 + q, "rlk-e")),
                       mask=W.zero_sum_mask(n, ctx.t, 80 + q) if q != 1 else None))
    d = [dict(cts=to_dev(q["cts"]), rlk=to_dev(q["rlk"]), mask=None if q["mask"] is None else to_dev(q["mask"]))
         for q in qs]
    outs = [empty((2, L, n), np.uint64) for _ in qs]
    sv.eval_batch([x["cts"] for x in d], [x["rlk"] for x in d], [x["mask"] for x in d], outs)
    for i, x in enumerate(d):
        alone = empty((2, L, n), np.uint64)
        sv.eval(x["cts"], x["rlk"], x["mask"], alone)
        got = to_host(outs[i], np.uint64)
        assert (to_host(alone, np.uint64) == got).all(), f"query {i}"
        assert (got == ctx.server_eval(qs[i]["cts"], spos, qs[i]["rlk"], 3, mask=qs[i]["mask"])).all()
        if qs[i]["mask"] is not None:
            assert PR.extract_cardinality(ctx.decrypt_slots(qs[i]["sk"], got)) == 0
    out = empty((2, L, n), np.uint64)
    for b0, b1 in [(0, 0), (1, 1), (0, gp.mu)]:
        sv.eval_range(to_dev(cts), to_dev(rlk), b0, b1, False, None, out)
        say(f"empty server range [{b0}, {b1})")
        assert (to_host(out, np.uint64) == 0).all()
