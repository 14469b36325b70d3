"""GPU parity of the single evaluator steps against the oracle (bit-exact)."""
import numpy as np
import pytest

from gpu_util import empty, pair, say, to_dev, to_host
from oracle import params as P
from oracle.core import lib as olib
import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def brv(k, bits):
    return int(format(k, f"0{bits}b")[::-1], 2)


@pytest.mark.parametrize("log_n", [10, 12, 13, 14])
def test_primes_and_roots_follow_the_rule(log_n):
    say(f"primes log_n={log_n}")
    gp, _ = pair(log_n, 3)
    n = 1 << log_n
    assert gp.primes == P.select_primes(n, gp.L + gp.K)
    for i, q in enumerate(gp.primes):
        assert gp.info.psi[i] == P.primitive_root_2n(q, n)
    assert gp.info.psi_t == P.primitive_root_2n(P.T_PLAIN, n)
    assert gp.info.q_bits == int(np.prod([int(q) for q in gp.q_primes], dtype=object)).bit_length()


@pytest.mark.parametrize("log_n", [10, 11, 12, 13, 14])
def test_ntt_is_evaluation_at_roots_bit_reversed(log_n):
    say(f"ntt log_n={log_n}")
    gp, _ = pair(log_n, 2)
    n, np_ = gp.n, gp.L + gp.K
    rows = 2 * np_
    primes = [gp.primes[r % np_] for r in range(rows)]
    x = np.stack([W.rng(log_n * 100 + r, "ntt").integers(0, q, size=n, dtype=np.uint64)
                  for r, q in enumerate(primes)])
    x[0, :] = 0
    x[0, 1] = 1                                 # X -> psi^(2 brv(k) + 1)
    d = to_dev(x)
    gp.ntt(d, rows, 0, np_, inverse=False)
    got = to_host(d, np.uint64)
    for r in range(rows):
        q = primes[r]
        e = x[r].copy()
        olib().or_eval_fwd(e, n, q, gp.info.psi[r % np_])   # natural order
        want = e[[brv(k, log_n) for k in range(n)]]
        assert (got[r] == want).all(), f"row {r}"
    gp.ntt(d, rows, 0, np_, inverse=True)
    assert (to_host(d, np.uint64) == x).all()


@pytest.mark.parametrize("log_n", [10, 12, 13])
def test_batch_encoding(log_n):
    say(f"encode log_n={log_n}")
    gp, ctx = pair(log_n, 2)
    slots = W.rng(log_n, "slots").integers(0, ctx.t, size=(3, gp.n)).astype(np.uint32)
    ds = to_dev(slots)
    dp = empty((3, gp.n), np.uint32)
    gp.encode(ds, dp)
    polys = to_host(dp, np.uint32)
    for i in range(3):
        assert (polys[i] == ctx.encode(slots[i])).all()
    back = empty((3, gp.n), np.uint32)
    gp.decode(dp, back)
    assert (to_host(back, np.uint32) == slots).all()


@pytest.mark.parametrize("log_n,L", [(10, 2), (12, 2), (13, 4)])
def test_encrypt_keygen_decrypt_match_oracle(log_n, L):
    say(f"encrypt log_n={log_n} L={L}")
    gp, ctx = pair(log_n, L)
    n = gp.n
    sk = W.secret_key(n, 7)
    slots = W.rng(8, "slots").integers(0, ctx.t, size=(3, n)).astype(np.uint32)
    a = W.uniform_residues((3,), ctx.primes, n, 9, "enc-a")
    e = W.errors((3, n), 10, "enc-e")
    dct = empty((3, 2, L, n), np.uint64)
    gp.encrypt(to_dev(sk), to_dev(slots), to_dev(a), to_dev(e), dct)
    got = to_host(dct, np.uint64)
    want = ctx.encrypt_many(sk, ctx.encode_many(slots), a, e)
    assert (got == want).all()
    ka = W.uniform_residues((L,), ctx.primes, n, 11, "rlk-a")
    ke = W.errors((L, n), 12, "rlk-e")
    drlk = empty((L, 2, L, n), np.uint64)
    gp.keygen_relin(to_dev(sk), to_dev(ka), to_dev(ke), drlk)
    assert (to_host(drlk, np.uint64) == ctx.keygen_relin(sk, ka, ke)).all()
    dslots = empty((3, n), np.uint32)
    gp.decrypt(to_dev(sk), to_dev(want), dslots)
    assert (to_host(dslots, np.uint32) == slots).all()
    assert gp.noise_budget(to_dev(sk), to_dev(want[0])) == ctx.noise_budget(sk, want[0])


def _fresh(ctx, sk, seed, count=2):
    n = ctx.n
    slots = W.rng(seed, "slots").integers(0, ctx.t, size=(count, n)).astype(np.uint32)
    a = W.uniform_residues((count,), ctx.primes, n, seed, "enc-a")
    e = W.errors((count, n), seed, "enc-e")
    return ctx.encrypt_many(sk, ctx.encode_many(slots), a, e), slots


@pytest.mark.parametrize("log_n,L", [(10, 2), (10, 3), (12, 2), (13, 4)])
def test_multiply_and_relin_match_oracle(log_n, L):
    say(f"multiply log_n={log_n} L={L}")
    gp, ctx = pair(log_n, L)
    n = gp.n
    sk = W.secret_key(n, 20)
    cts, slots = _fresh(ctx, sk, 21)
    d3 = empty((3, L, n), np.uint64)
    gp.multiply(to_dev(cts[0]), to_dev(cts[1]), d3)
    got3 = to_host(d3, np.uint64)
    want3 = ctx.multiply(cts[0], cts[1])
    assert (got3 == want3).all()
    rlk = ctx.keygen_relin(sk, W.uniform_residues((L,), ctx.primes, n, 22, "rlk-a"), W.errors((L, n), 23, "rlk-e"))
    d2 = empty((2, L, n), np.uint64)
    gp.relin(to_dev(want3), to_dev(rlk), d2)
    got2 = to_host(d2, np.uint64)
    assert (got2 == ctx.relin(want3, rlk)).all()
    assert (ctx.decrypt_slots(sk, got2) == slots[0].astype(np.int64) * slots[1] % ctx.t).all()


@pytest.mark.parametrize("L", [2, 3])
def test_rounding_ties_take_the_exact_path(L):
    """Inputs whose centred lift or rescale lies within 2^-200 of a rounding tie."""
    say(f"exact path L={L}")
    gp, ctx = pair(10, L)
    n, Q, t = gp.n, ctx.Q, ctx.t
    half_lo, half_hi = (Q - 1) // 2, (Q + 1) // 2
    tinv = pow(t, -1, Q)
    cases = [
        (half_lo, 1), (half_hi, 1), (half_hi, half_hi), (half_lo, half_lo),
        (1, tinv * half_hi % Q), (1, tinv * half_lo % Q), (Q - 1, tinv * half_hi % Q),
    ]
    before = gp.exact_path_count()
    for alpha, beta in cases:
        x = np.zeros((2, L, n), np.uint64)
        y = np.zeros((2, L, n), np.uint64)
        x[0] = ctx.ints_to_poly([alpha] + [0] * (n - 1))
        y[0] = ctx.ints_to_poly([beta] + [0] * (n - 1))
        x[1] = ctx.ints_to_poly([alpha] * n)          # a full polynomial of near-tie values
        y[1] = ctx.ints_to_poly([beta] * n)
        d3 = empty((3, L, n), np.uint64)
        gp.multiply(to_dev(x), to_dev(y), d3)
        assert (to_host(d3, np.uint64) == ctx.multiply(x, y)).all(), (alpha, beta)
    assert gp.exact_path_count() > before


def test_select_sum_matches_oracle():
    say("select-sum")
    gp, ctx = pair(10, 2, h=3, item_bits=10)
    n, ell, h = gp.n, gp.ell, gp.h
    sk = W.secret_key(n, 30)
    planes = W.planes_random(ell, n, 31)
    cts = ctx.encrypt_many(sk, ctx.encode_many(planes), W.uniform_residues((ell,), ctx.primes, n, 32, "a"),
                           W.errors((ell, n), 33, "e"))
    from oracle import cw as CW
    import math
    vals = W.rng(34, "cw").integers(0, math.comb(ell, h), size=n)
    pos = CW.encode_many(vals, ell, h)
    pos[5] = CW.NO_POS
    out = empty((2, gp.L, n), np.uint64)
    gp.select_sum(to_dev(cts), to_dev(pos), out)
    assert (to_host(out, np.uint64) == ctx.select_sum(cts, pos, h)).all()


def test_issue_rate_probes_are_plausible():
    """The measured instruction rates that set the VALU and matrix rooflines: positive, and not
    above what the chip can issue (256 CUs x 64 lanes at up to 2.4 GHz, two VALU operations per
    lane per clock for the simplest ones, and the published 5.0 POP/s dense int8 matrix peak, each
    with 20% headroom)."""
    say("issue-rate probes")
    import paper_2310_14565_amd as pk
    lane_issue = 256 * 64 * 2.4e9
    for kind, name in enumerate(pk.VALU_KINDS):
        r = pk.probe_valu(kind)
        assert 0.01 * lane_issue < r < 2.4 * lane_issue, (name, r)
    m = pk.probe_mfma_int8()
    assert 0.1 * 5.0e15 < m < 1.2 * 5.0e15, m
    with pytest.raises(Exception):
        pk.probe_valu(7)
