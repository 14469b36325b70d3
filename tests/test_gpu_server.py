"""GPU parity of the whole server computation (Alg. 1 + 2 / 5) against the oracle."""
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


def run_case(log_n, L, h, item_bits, n_server, m_client, planted, mu=None, seed=1, cache=False,
             mask=True, check_full=True):
    import paper_2310_14565_amd as pk
    n = 1 << log_n
    mu = mu or P.server_bin_bound(n_server, n)
    cfg = PR.Config(n=n, L=L, h=h, item_bits=item_bits, mu=mu)
    gp = pk.Params(log_n, L, h, item_bits, mu, hash_seed=cfg.hash_seed)
    ctx = Context(n, gp.q_primes)
    assert gp.ell == cfg.ell
    server = W.server_items(n_server, item_bits, seed)
    client = W.client_items(m_client, server, planted, item_bits, seed + 1)
    # client side: library host preparation equals the oracle's
    ctab, cval, _, planes = PR.client_prepare(cfg, client)
    gtab, gval = gp.client_table(client)
    assert (gtab == ctab).all() and (gval == cval).all()
    assert (gp.codeword_planes(gtab, gval) == planes).all()
    stab, sval, spos, max_load = PR.server_prepare(cfg, server)
    sk = W.secret_key(n, seed + 2)
    rlk = ctx.keygen_relin(sk, W.uniform_residues((L,), ctx.primes, n, seed + 3, "rlk-a"),
                           W.errors((L, n), seed + 3, "rlk-e"))
    cts = PR.encrypt_planes(ctx, sk, planes, W.uniform_residues((cfg.ell,), ctx.primes, n, seed + 4, "enc-a"),
                            W.errors((cfg.ell, n), seed + 4, "enc-e"))
    m = W.zero_sum_mask(n, ctx.t, seed + 5) if mask else None
    say(f"server log_n={log_n} L={L} h={h} ell={cfg.ell} mu={mu} max_load={max_load} cache={cache}")
    sv = pk.Server(gp, server, cache_plaintexts=cache)
    assert sv.max_load == max_load
    assert (sv.codewords() == spos).all()
    out = empty((2, L, n), np.uint64)
    sv.eval(to_dev(cts), to_dev(rlk), None if m is None else to_dev(m), out)
    got = to_host(out, np.uint64)
    if check_full:
        want = ctx.server_eval(cts, spos, rlk, h, mask=m)
        assert (got == want).all()
    slots = ctx.decrypt_slots(sk, got)
    if mask:
        assert PR.extract_cardinality(slots) == planted
    else:
        assert (slots == PR.plaintext_membership(ctab, cval, stab, sval)).all()
    assert ctx.noise_budget(sk, got) > 0
    return gp, ctx, sv, cts, rlk, spos, sk


@pytest.mark.parametrize("h,item_bits", [(1, 9), (2, 10), (3, 12), (4, 12)])
def test_small_product_trees(h, item_bits):
    run_case(10, 3, h, item_bits, n_server=200, m_client=40, planted=9, seed=10 + h)


def test_indicator_mode():
    run_case(10, 3, 2, 10, n_server=300, m_client=50, planted=17, seed=40, mask=False)


@pytest.mark.parametrize("cache", [False, True])
def test_toy_configuration(cache):
    """N=4096, two primes, h=2, l=363, 256 server / 16 client 16-bit items, 4 planted."""
    run_case(12, 2, 2, 16, n_server=256, m_client=16, planted=4, mu=P.server_mu(256, 4096),
             seed=11, cache=cache)


def test_eval_range_sums_to_the_whole():
    gp, ctx, sv, cts, rlk, spos, sk = run_case(10, 3, 2, 10, n_server=300, m_client=50, planted=17, seed=50)
    L, n = gp.L, gp.n
    acc = np.zeros((2, L, n), dtype=object)
    for b0, b1 in [(0, 2), (2, 3), (3, gp.mu)]:
        out = empty((2, L, n), np.uint64)
        sv.eval_range(to_dev(cts), to_dev(rlk), b0, b1, False, None, out)
        part = to_host(out, np.uint64)
        assert (part == ctx.server_eval(cts, spos, rlk, gp.h, finalize=False, begin=b0, end=b1)).all()
        acc += part.astype(object)
    for l, q in enumerate(ctx.primes):
        acc[:, l] %= q
    whole = ctx.server_eval(cts, spos, rlk, gp.h, finalize=False)
    assert (acc.astype(np.uint64) == whole).all()
