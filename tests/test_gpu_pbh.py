"""GPU parity with permutation-based hashing (Sec. 3.3): host tables, the whole server
computation for h = 2 and h = 8 (three tree levels), and the paper's own 32-bit parameters
(b = N = 8192, h = 8, n = 2^20) at full size on sampled batches."""
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


@pytest.mark.parametrize("h,L,item_bits,cache", [(2, 3, 20, False), (8, 4, 22, True), (3, 4, 18, True)])
def test_pbh_server_matches_oracle(h, L, item_bits, cache):
    import paper_2310_14565_amd as pk
    log_n = 10
    n = 1 << log_n
    n_server, m_client, planted, seed = 700, 120, 23, 90 + h
    mu = P.server_bin_bound(n_server, n)
    cfg = PR.Config(n=n, L=L, h=h, item_bits=item_bits, mu=mu, pbh=True)
    gp = pk.Params(log_n, L, h, item_bits, mu, hash_seed=cfg.hash_seed, pbh=True)
    assert gp.ell == cfg.ell and gp.effective_bits == cfg.effective_bits and gp.pbh
    ctx = Context(n, gp.q_primes)
    server = W.server_items(n_server, item_bits, seed)
    client = W.client_items(m_client, server, planted, item_bits, seed + 1)
    ctab, cval, _, planes = PR.client_prepare(cfg, client)
    gtab, gval = gp.client_table(client)
    assert (gtab == ctab).all() and (gval == cval).all()
    assert (gp.codeword_planes(gtab, gval) == planes).all()
    stab, sval, spos, max_load = PR.server_prepare(cfg, server)
    sv = pk.Server(gp, server, cache_plaintexts=cache)
    assert sv.max_load == max_load and (sv.codewords() == spos).all()
    sk = W.secret_key(n, seed + 2)
    rlk = ctx.keygen_relin(sk, W.uniform_residues((L,), ctx.primes, n, seed + 3, "rlk-a"),
                           W.errors((L, n), seed + 3, "rlk-e"))
    cts = PR.encrypt_planes(ctx, sk, planes, W.uniform_residues((cfg.ell,), ctx.primes, n, seed + 4, "enc-a"),
                            W.errors((cfg.ell, n), seed + 4, "enc-e"))
    mask = W.zero_sum_mask(n, ctx.t, seed + 5)
    say(f"pbh h={h} L={L} ell={cfg.ell} lambda_bar={cfg.effective_bits} max_load={max_load}")
    out = empty((2, L, n), np.uint64)
    sv.eval(to_dev(cts), to_dev(rlk), to_dev(mask), out)
    got = to_host(out, np.uint64)
    assert (got == ctx.server_eval(cts, spos, rlk, h, mask=mask)).all()
    assert PR.extract_cardinality(ctx.decrypt_slots(sk, got)) == planted
    assert ctx.noise_budget(sk, got) > 0
    sv.eval(to_dev(cts), to_dev(rlk), None, out)
    ind = ctx.decrypt_slots(sk, to_host(out, np.uint64))
    assert (ind == PR.plaintext_membership(ctab, cval, stab, sval)).all()


@pytest.mark.slow
@pytest.mark.timeout(600)
def test_paper_32bit_parameters_full_size():
    """b = N = 8192, h = 8, lambda = 32 with PBH (lambda_bar = 21, l = 27), L = 4, n = 2^20,
    mu = 526: one sampled batch against the oracle, and an encrypted query of m = 1024."""
    import torch
    import bench
    import paper_2310_14565_amd as pk
    n, L, h, mu = 8192, 4, 8, 526
    cfg = PR.Config(n=n, L=L, h=h, item_bits=32, mu=mu, pbh=True)
    gp = pk.Params(13, L, h, 32, mu, pbh=True)
    assert gp.ell == cfg.ell == 27
    ctx = Context(n, gp.q_primes)
    items = W.server_items(1 << 20, 32, 51)
    sv = pk.Server(gp, items, cache_plaintexts=True)
    _, _, spos, max_load = PR.server_prepare(cfg, items)
    assert sv.max_load == max_load and (sv.codewords() == spos).all()
    cts = W.uniform_residues((gp.ell, 2), ctx.primes, n, 52, "pbh-cts")
    rlk = W.uniform_residues((L, 2), ctx.primes, n, 53, "pbh-rlk")
    out = empty((2, L, n), np.uint64)
    b = max_load - 1
    sv.eval_range(to_dev(cts), to_dev(rlk), b, b + 1, False, None, out)
    assert (to_host(out, np.uint64) == ctx.server_eval(cts, spos, rlk, h, finalize=False, begin=b, end=b + 1)).all()
    q = bench.make_query(gp, items, {"item_bits": 32}, 1024, 256, 54)
    res = torch.zeros((2, L, n), dtype=torch.int64, device="cuda")
    sv.eval(q["cts"], q["rlk"], q["mask"], res)
    slots = torch.zeros((1, n), dtype=torch.int32, device="cuda")
    gp.decrypt(q["sk"], res.reshape(1, 2, L, n), slots)
    assert int(to_host(slots, np.uint32).astype(np.int64).sum() % 65537) == 256
    assert gp.noise_budget(q["sk"], res) > 0
    sv.close()
