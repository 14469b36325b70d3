"""Large elements on the GPU (Sec. 5 "Optimization for Large Elements"; Sec. 7 "Parameters for
Large Elements"): byte strings hashed to lambda = 40 + ceil(log2(b mu)) bits, permutation-based
hashing, a weight-16 code over the stored bits, through the 64-bit C-ABI calls.  Every result
equals the oracle's bit for bit, for PSI-cardinality and PSI-Sum, alone and batched."""
import numpy as np
import pytest

from gpu_util import empty, say, to_dev, to_host
from oracle import large as LG, params as P, protocol as PR
from oracle.core import Context
import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _query(ctx, cfg, hc, seed):
    _, _, _, planes = PR.client_prepare(cfg, hc)
    sk = W.secret_key(ctx.n, seed)
    rlk = ctx.keygen_relin(sk, W.uniform_residues((ctx.L,), ctx.primes, ctx.n, seed + 1, "rlk-a"),
                           W.errors((ctx.L, ctx.n), seed + 1, "rlk-e"))
    cts = PR.encrypt_planes(ctx, sk, planes, W.uniform_residues((cfg.ell,), ctx.primes, ctx.n, seed + 2, "enc-a"),
                            W.errors((cfg.ell, ctx.n), seed + 2, "enc-e"))
    return sk, rlk, cts


@pytest.mark.parametrize("with_values", [False, True])
def test_hashed_elements_match_oracle(with_values):
    import paper_2310_14565_amd as pk
    log_n, L, h, n_server = 10, 5, 16, 1500
    n = 1 << log_n
    mu = P.server_bin_bound(n_server, n)
    lam = pk.large_element_bits(n, 1, mu)
    assert lam == LG.element_bits(n, 1, mu) and lam > 32
    cfg = PR.Config(n=n, L=L, h=h, item_bits=lam, mu=mu, pbh=True)
    gp = pk.Params(log_n, L, h, lam, mu, hash_seed=cfg.hash_seed, pbh=True)
    assert gp.wide and gp.ell == cfg.ell and gp.effective_bits == cfg.effective_bits
    ctx = Context(n, gp.q_primes)
    server_e = LG.random_elements(n_server, 32, 31)
    hs = pk.hash_elements(server_e, lam)
    assert (hs == LG.hash_elements(server_e, lam)).all()
    values = W.item_values(n_server, 1, 1 << 12, 32) if with_values else None
    sv = pk.Server(gp, hs, cache_plaintexts=True, values=values)
    _, _, spos, _ = PR.server_prepare(cfg, hs)
    assert (sv.codewords() == spos).all()
    say(f"large elements: lambda={lam} lambda_bar={gp.effective_bits} ell={gp.ell} max_load={sv.max_load} "
        f"planes={sv.plane_groups}")
    vals = PR.server_values(cfg, hs, values) if with_values else None
    queries = []
    for q, planted in enumerate((9, 3)):
        client_e = server_e[100 * q:100 * q + planted] + LG.random_elements(40 - planted, 32, 33 + q,
                                                                             exclude=server_e)
        hc = pk.hash_elements(client_e, lam)
        table, valid = gp.client_table(hc)
        otable, ovalid, _, _ = PR.client_prepare(cfg, hc)
        assert (table == otable).all() and (valid == ovalid).all()
        sk, rlk, cts = _query(ctx, cfg, hc, 40 + 10 * q)
        mask = W.zero_sum_mask(n, ctx.t, 60 + q)
        want = ctx.server_eval(cts, spos, rlk, h, mask=mask, vals=vals)
        queries.append(dict(sk=sk, rlk=rlk, cts=cts, mask=mask, want=want, planted=planted,
                            common=list(range(100 * q, 100 * q + planted))))
    d = [dict(cts=to_dev(x["cts"]), rlk=to_dev(x["rlk"]), mask=to_dev(x["mask"])) for x in queries]
    for x, dd in zip(queries, d):
        out = empty((2, L, n), np.uint64)
        sv.eval(dd["cts"], dd["rlk"], dd["mask"], out)
        got = to_host(out, np.uint64)
        assert (got == x["want"]).all()
        slots = ctx.decrypt_slots(x["sk"], got)
        if with_values:
            assert PR.extract_sum(slots) == int(values[x["common"]].astype(np.int64).sum() % ctx.t)
        else:
            assert PR.extract_cardinality(slots) == x["planted"]
        assert ctx.noise_budget(x["sk"], got) > 0
    outs = [empty((2, L, n), np.uint64) for _ in d]
    sv.eval_batch([x["cts"] for x in d], [x["rlk"] for x in d], [x["mask"] for x in d], outs)
    for x, o in zip(queries, outs):
        assert (to_host(o, np.uint64) == x["want"]).all()
    sv.close()
