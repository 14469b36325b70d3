#!/usr/bin/env python3
"""Benchmark of the PEPSI PSI-cardinality server computation on one MI355X.

Workload (the paper-shaped single query, plain path): N = 8192 bins/slots,
L = 4 ciphertext primes (216-bit Q), t = 65537, Hamming weight h = 4, code
length 569 (32-bit elements, eq. (1)), server maximum bin load mu = 526 (the
paper's value for n = 2^20, b = 8192), server set n = 2^20 random 32-bit
items, client set m = 1024 with 256 planted common items; cardinality output
with a zero-sum mask.  Synthetic seeded data (workload/).

A step is one server evaluation of one client request (every step of the
path: client-ciphertext NTTs, select-and-sum over all server batches, the
equality product with relinearisation, accumulation, (h!)^-1, mask, inverse
NTT), with the request, relinearisation key and the server's prepared set
resident in HBM.  The metric counts slot comparisons b * mu per query
(Arith-CW-Eq evaluations between a client bin entry and a server bin entry,
dummies included).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CONFIGS = {
    # log_n, L, h, item_bits, mu, n_server, m_client, planted
    "paper": dict(log_n=13, L=4, h=4, item_bits=32, mu=526, n_server=1 << 20, m_client=1024, planted=256),
    "toy": dict(log_n=12, L=2, h=2, item_bits=16, mu=11, n_server=256, m_client=16, planted=4),
    # large: the server plaintexts (2.1 TB) cannot be resident; run with --mode generate
    "large": dict(log_n=14, L=8, h=4, item_bits=32, mu=3487, n_server=1 << 24, m_client=4096, planted=1024),
}
# Serving workload: a resident n = 2^22 set at N = 8192, mu = 1870 (the least mu with
# b * P[Bin(3n, 1/b) >= mu] <= 2^-40), requests with m log-uniform in [128, 4096], 25% planted,
# Poisson arrivals at 0.8 x the measured saturated capacity.
SERVE = dict(log_n=13, L=4, h=4, item_bits=32, mu=1870, n_server=1 << 22, m_lo=128, m_hi=4096)
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a: np.ndarray):
    import torch
    a = np.ascontiguousarray(a)
    view = {8: np.int64, 4: np.int32, 2: np.int16, 1: np.int8}[a.dtype.itemsize]
    return torch.from_numpy(a.view(view).copy()).cuda()


def select_sum_source_digest() -> str:
    """SHA-256 of the select-and-sum kernel's source (its constants, helper, kernel body and launcher):
    hardware byte counts taken for one version of the kernel are void for any other."""
    src = open(os.path.join(ROOT, "paper_2310_14565_amd", "csrc", "rns.hip")).read()
    a = src.index("constexpr int IB = ")
    z = src.index("// Select-and-sum of several queries")
    la = src.index("void select_sum(const Tables& T")
    lz = src.index("\n}\n", la) + 3
    return hashlib.sha256((src[a:z] + src[la:lz]).encode()).hexdigest()


def traffic_record(kernel: str):
    """HBM traffic from committed rocprofv3 counter runs, if they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        if rec.get("source_sha256") != select_sum_source_digest():
            return None
    except (OSError, ValueError):
        return None
    return rec


# The lazy Shoup butterfly on 32-bit lanes (the NTT's per-butterfly minimum): the truncated quotient
# takes two high 32 x 32 products and one 32 x 32 -> 64 multiply-add, the low 64 bits of x w - q p two
# multiply-adds and four low products, and the sums (two three-input adds, one add, U + V, U - V + 4p)
# eight single-issue operations.
BUTTERFLY_MIX = {"v_mad_u64_u32": 3, "v_mul_hi_u32": 2, "v_mul_lo_u32": 4, "v_add_u32": 8}
CHIP_LANE_ISSUE = 256 * 64 * 2.4e9          # 256 CUs x 64 lanes x 2.4 GHz, one VALU op per lane per clock
PRODUCT_MADS = 3                             # v_mad_u64_u32 per exact 54-bit product (27-bit halves)
MFMA_DIGIT_PAIRS = 7 * 7                     # balanced int8 digits per 54-bit residue, squared
INT8_DENSE_PEAK_T = 5000.0                   # MI355X dense int8 matrix peak, TOP/s


def valu_roofline(pk, tm, n):
    """Integer-VALU roofline of the transforms, rescales and extensions: measured issue rates of
    their instructions (pepsi_probe_valu) give the peak butterfly and modular-product rates; the
    engine's event-timed launches of the timed steps give the achieved ones."""
    rates = {k: pk.probe_valu(i) for i, k in enumerate(pk.VALU_KINDS)}
    sec_per_bfly = sum(cnt / rates[k] for k, cnt in BUTTERFLY_MIX.items())   # per lane, whole chip
    peak = 1.0 / sec_per_bfly
    logn = n.bit_length() - 1
    out = {"valu_probe_T_lane_ops_per_s": {k: round(v / 1e12, 3) for k, v in rates.items()},
           "chip_lane_issue_T_per_s": round(CHIP_LANE_ISSUE / 1e12, 2),
           "butterfly_mix": BUTTERFLY_MIX}
    for name, rows, ms, launches in (("k_ntt_fwd", tm.ntt_fwd_rows, tm.ntt_fwd_ms, tm.ntt_fwd_launches),
                                     ("k_ntt_inv", tm.ntt_inv_rows, tm.ntt_inv_ms, tm.ntt_inv_launches)):
        if not launches or ms <= 0:
            continue
        bfly = rows * (n // 2) * logn
        achieved = bfly / (ms / 1e3)
        out[name] = {"bound": "alu", "achieved": round(achieved / 1e9, 1), "peak": round(peak / 1e9, 1),
                     "unit": "Gbutterfly/s", "frac": round(achieved / peak, 4),
                     "avg_launch_ms": round(ms / launches, 4), "rows_per_launch": round(rows / launches, 1),
                     "ns_per_row": round(1e6 * ms / rows, 2)}
    # The exact rescales and Q -> B extensions, in 54-bit modular products (pepsi_timing): each
    # costs at least three v_mad_u64_u32 (27-bit halves into 64-bit accumulators), so the peak is
    # a third of that instruction's measured rate.
    peak_prod = rates["v_mad_u64_u32"] / PRODUCT_MADS
    out["product_mix"] = {"v_mad_u64_u32": PRODUCT_MADS}
    for name, prods, ms, launches in (("k_scale_round", tm.rescale_products, tm.rescale_ms, tm.rescale_launches),
                                      ("k_ext_q_to_b", tm.ext_products, tm.ext_ms, tm.ext_launches)):
        if not launches or ms <= 0:
            continue
        achieved = prods / (ms / 1e3)
        out[name] = {"bound": "alu", "achieved": round(achieved / 1e9, 1), "peak": round(peak_prod / 1e9, 1),
                     "unit": "G modular products/s", "frac": round(achieved / peak_prod, 4),
                     "avg_launch_ms": round(ms / launches, 4),
                     "products_per_launch": int(prods / launches)}
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, params, server_items, seed, computed_batches):
    """The oracle timed on a bounded sample: the client-ciphertext transforms, then four server
    batches spread over the batches that hold items (each timed alone), extrapolated linearly to
    one query over all mu batches (the oracle computes every batch, dummies included)."""
    from oracle import protocol as PR
    from oracle.core import Context, num_threads
    import workload as W
    n, L, h = 1 << cfg["log_n"], cfg["L"], cfg["h"]
    ctx = Context(n, params.q_primes)
    pcfg = PR.Config(n=n, L=L, h=h, item_bits=cfg["item_bits"], mu=cfg["mu"])
    _, _, spos, _ = PR.server_prepare(pcfg, server_items)
    ell = pcfg.ell
    cts = W.uniform_residues((ell, 2), ctx.primes, n, seed, "cpu-cts")
    rlk = W.uniform_residues((L, 2), ctx.primes, n, seed, "cpu-rlk")
    t0 = time.perf_counter()
    ctx.server_eval(cts, spos, rlk, h, finalize=False, begin=0, end=0)
    t_prep = time.perf_counter() - t0
    sample = sorted({0, computed_batches // 3, (2 * computed_batches) // 3, max(computed_batches - 1, 0)})
    per = []
    for b in sample:
        t0 = time.perf_counter()
        ctx.server_eval(cts, spos, rlk, h, finalize=False, begin=b, end=b + 1)
        per.append(max(time.perf_counter() - t0 - t_prep, 1e-9))
    t_batch = float(np.mean(per))
    t_query = t_prep + cfg["mu"] * t_batch
    return {
        "value": n * cfg["mu"] / t_query,
        "unit": "slot-comparisons/s",
        "cores": num_threads(),
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "nproc": len(os.sched_getaffinity(0)),
        "sample": (f"client-ciphertext transforms ({t_prep:.2f} s) + server batches {sample} of {cfg['mu']} timed "
                   f"one by one ({', '.join(f'{x:.2f}' for x in per)} s), their mean extrapolated linearly to one "
                   f"query ({t_query:.0f} s)"),
    }


def make_query(params, server_items, cfg, m, planted, seed):
    """One client request on the GPU: host hashing/encoding, GPU encryption with its own key."""
    import torch
    import workload as W
    n, L, ell = params.n, params.L, params.ell
    client = W.client_items(m, server_items, planted, cfg["item_bits"], seed)
    table, valid = params.client_table(client)
    planes = params.codeword_planes(table, valid)
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    sk = dev(W.secret_key(n, seed + 1))
    a = torch.stack([torch.randint(0, q, (ell, n), generator=g, device="cuda", dtype=torch.int64)
                     for q in params.q_primes], dim=1).contiguous()
    e = torch.clamp(torch.round(torch.randn((ell, n), generator=g, device="cuda") * 3.2), -19, 19).to(torch.int32)
    cts = torch.empty((ell, 2, L, n), dtype=torch.int64, device="cuda")
    params.encrypt(sk, dev(planes), a, e, cts)
    ka = torch.stack([torch.randint(0, q, (L, n), generator=g, device="cuda", dtype=torch.int64)
                      for q in params.q_primes], dim=1).contiguous()
    ke = torch.clamp(torch.round(torch.randn((L, n), generator=g, device="cuda") * 3.2), -19, 19).to(torch.int32)
    rlk = torch.empty((L, 2, L, n), dtype=torch.int64, device="cuda")
    params.keygen_relin(sk, ka, ke, rlk)
    mask = dev(W.zero_sum_mask(n, 65537, seed + 2))
    return dict(sk=sk, cts=cts, rlk=rlk, mask=mask, planted=planted, m=m, client=client)


def serving_leg(pk, requests, pool, slots, load, seed, planes_only=False):
    """Continuous batching: `requests` requests over a pool of distinct client queries, Poisson arrivals
    at `load` x the saturated capacity measured first on the same handle; latency = completion minus
    scheduled arrival."""
    import torch
    import workload as W
    sc = SERVE
    n, L = 1 << sc["log_n"], sc["L"]
    params = pk.Params(sc["log_n"], L, sc["h"], sc["item_bits"], sc["mu"])
    server_items = W.server_items(sc["n_server"], sc["item_bits"], seed)
    g = W.rng(seed, "serve-sizes")
    sizes = np.rint(np.exp(g.uniform(np.log(sc["m_lo"]), np.log(sc["m_hi"]), size=pool))).astype(int)
    log(f"[bench] serving leg: n={sc['n_server']} mu={sc['mu']}, pool of {pool} queries, m in "
        f"[{sizes.min()}, {sizes.max()}]")
    qs = [make_query(params, server_items, sc, int(m), int(round(0.25 * m)), seed + 100 * (i + 1))
          for i, m in enumerate(sizes)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    server = pk.Server(params, server_items, cache_plaintexts=True, planes_only=planes_only)
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t0
    log(f"[bench] serving server ready in {prep_s:.1f} s: max load {server.max_load}, "
        f"{server.cached_batches} of {server.max_load} batches cached, {server.plane_groups} digit-plane groups")
    outs = [torch.zeros((2, L, n), dtype=torch.int64, device="cuda") for _ in range(requests)]
    torch.cuda.synchronize()
    free_b, _ = torch.cuda.mem_get_info()
    budget = max(free_b - (2 << 30), 0)          # admission by memory: what is left beside a 2 GiB reserve
    srv = pk.Serve(server, max_active=slots, hbm_budget=budget)
    slots = srv.info().slots
    log(f"[bench] serving: HBM budget {budget / 2**30:.1f} GiB, {srv.info().slot_bytes / 2**20:.0f} MiB per slot, "
        f"{slots} slots")

    def submit(i):
        q = qs[i % pool]
        return srv.submit(q["cts"], q["rlk"], q["mask"], outs[i])

    # saturated capacity: one full set of slots at once
    c0 = pk.clock()
    ids = [submit(i) for i in range(slots)]
    st = [srv.wait(r) for r in ids]
    capacity = slots / (max(s.done_s for s in st) - c0)
    rate = load * capacity
    log(f"[bench] saturated capacity {capacity:.2f} queries/s; arrivals at {rate:.2f}/s")
    arrivals = np.cumsum(W.rng(seed, "serve-arrivals").exponential(1.0 / rate, size=requests))
    ids = []
    c0 = pk.clock()
    for i in range(requests):
        while pk.clock() < c0 + arrivals[i]:
            time.sleep(min(0.002, max(0.0, c0 + arrivals[i] - pk.clock())))
        ids.append(submit(i))
        if (i + 1) % 100 == 0:
            log(f"[bench] submitted {i + 1}/{requests}, completed {srv.info().completed - slots}")
    st = [srv.wait(r) for r in ids]
    info = srv.info()
    srv.close()
    lat = np.array([s.done_s - (c0 + a) for s, a in zip(st, arrivals)])
    span = max(s.done_s for s in st) - c0
    # every request decrypts to its planted cardinality, and repeats of one query are bit-identical
    bad = 0
    first = {}
    for i in range(requests):
        k = i % pool
        if k in first:
            bad += not torch.equal(outs[i], outs[first[k]])
            continue
        first[k] = i
        slots_t = torch.zeros((1, n), dtype=torch.int32, device="cuda")
        params.decrypt(qs[k]["sk"], outs[i].reshape(1, 2, L, n), slots_t)
        torch.cuda.synchronize()
        bad += int(slots_t.cpu().numpy().view(np.uint32).astype(np.int64).sum() % 65537) != qs[k]["planted"]
    if bad:
        log(f"[bench] WRONG RESULT in {bad} served requests")
        sys.exit(1)
    max_load, cached_batches, plane_groups = server.max_load, server.cached_batches, server.plane_groups
    server.close()
    comparisons = n * sc["mu"]
    return {
        "workload": (f"N={n} L={L} h={sc['h']} ell={params.ell} n={sc['n_server']} mu={sc['mu']}, "
                     f"m log-uniform [{sc['m_lo']}, {sc['m_hi']}], 25% planted"),
        "requests": requests,
        "query_pool": pool,
        "slots": info.slots,
        "hbm_budget_bytes": int(budget),
        "slot_bytes": int(info.slot_bytes),
        "tiles_per_cycle": info.tiles,
        "store": "digit planes only" if planes_only else "NTT-form cache (+ digit planes when both fit)",
        "cached_batches": int(cached_batches),
        "plane_groups": int(plane_groups),
        "server_max_load": int(max_load),
        "batches_computed": int(max_load),
        "value_computed_batches": round(requests * n * max_load / span, 1),
        "saturated_queries_per_s": round(capacity, 3),
        "arrival_rate_per_s": round(rate, 3),
        "queries_per_s": round(requests / span, 3),
        "value": round(requests * comparisons / span, 1),
        "unit": "slot-comparisons/s",
        "latency_ms": {"p50": round(1e3 * float(np.percentile(lat, 50)), 1),
                       "p99": round(1e3 * float(np.percentile(lat, 99)), 1),
                       "max": round(1e3 * float(lat.max()), 1)},
        "prep_s": round(prep_s, 2),
        "checked": "cardinality of every pool query; repeats bit-identical",
    }


def compression_leg(params, response, seed):
    """Request sent as its c0 halves plus a 32-byte seed (the server expands the c1 halves with
    ChaCha20), response switched to one prime: sizes and the GPU time of both steps."""
    import torch
    import workload as W
    n, L, ell = params.n, params.L, params.ell
    key = bytes(W.rng(seed, "request-seed").integers(0, 256, 32, dtype=np.uint8))
    req = torch.empty((ell, 2, L, n), dtype=torch.int64, device="cuda")
    small = torch.empty((2, n), dtype=torch.int64, device="cuda")
    params.expand_uniform(key, 0, ell, req, out_stride=2 * L * n, offset_words=L * n)
    params.mod_switch(response, small)
    torch.cuda.synchronize()
    a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    a.record()
    for _ in range(5):
        params.expand_uniform(key, 0, ell, req, out_stride=2 * L * n, offset_words=L * n)
    b.record()
    for _ in range(5):
        params.mod_switch(response, small)
    c.record()
    torch.cuda.synchronize()
    del req
    return {
        "request_bytes": ell * 2 * L * n * 8,
        "compressed_request_bytes": ell * L * n * 8 + 32,
        "expand_ms": round(a.elapsed_time(b) / 5, 3),
        "response_bytes": 2 * L * n * 8,
        "switched_response_bytes": 2 * n * 8,
        "mod_switch_ms": round(b.elapsed_time(c) / 5, 4),
    }


def psi_sum_leg(pk, params, server_items, cfg, steps, seed):
    """PSI-Sum (Alg. 5) on the same workload: server values uniform 12-bit, plaintexts cached."""
    import torch
    import workload as W
    n, L = params.n, params.L
    values = W.item_values(server_items.shape[0], 0, 1 << 12, seed)
    server = pk.Server(params, server_items, cache_plaintexts=True, values=values)
    q = make_query(params, server_items, cfg, cfg["m_client"], cfg["planted"], seed + 1)
    out = torch.zeros((2, L, n), dtype=torch.int64, device="cuda")
    server.eval(q["cts"], q["rlk"], q["mask"], out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        server.eval(q["cts"], q["rlk"], q["mask"], out)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    slots = torch.zeros((1, n), dtype=torch.int32, device="cuda")
    params.decrypt(q["sk"], out.reshape(1, 2, L, n), slots)
    torch.cuda.synchronize()
    got = int(slots.cpu().numpy().view(np.uint32).astype(np.int64).sum() % 65537)
    common = np.isin(server_items, q["client"])
    want = int(values[common].astype(np.int64).sum() % 65537)
    server.close()
    if got != want:
        log(f"[bench] WRONG PSI-Sum: {got} (want {want})")
        sys.exit(1)
    return {
        "ms_per_query": round(1e3 * t, 3),
        "value": round(n * cfg["mu"] / t, 1),
        "unit": "slot-comparisons/s",
        "steps": steps,
        "check": {"sum_mod_t": got},
    }


def paper32_leg(pk, steps, seed):
    """The paper's own 32-bit parameters (Sec. 7): b = N = 8192, h = 8 with permutation-based
    hashing (stored values of 21 bits with the hash index, l = 27), L = 4, n = 2^20, m = 1024 with
    256 planted, mu = 526, plaintexts cached."""
    import torch
    import workload as W
    n, L = 8192, 4
    params = pk.Params(13, L, 8, 32, 526, pbh=True)
    items = W.server_items(1 << 20, 32, seed)
    t0 = time.perf_counter()
    server = pk.Server(params, items, cache_plaintexts=True)
    torch.cuda.synchronize()
    prep = time.perf_counter() - t0
    q = make_query(params, items, {"item_bits": 32}, 1024, 256, seed + 1)
    out = torch.zeros((2, L, n), dtype=torch.int64, device="cuda")
    server.eval(q["cts"], q["rlk"], q["mask"], out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        server.eval(q["cts"], q["rlk"], q["mask"], out)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    slots = torch.zeros((1, n), dtype=torch.int32, device="cuda")
    params.decrypt(q["sk"], out.reshape(1, 2, L, n), slots)
    torch.cuda.synchronize()
    card = int(slots.cpu().numpy().view(np.uint32).astype(np.int64).sum() % 65537)
    budget = params.noise_budget(q["sk"], out)
    server.close()
    if card != 256 or budget <= 0:
        log(f"[bench] WRONG RESULT with the paper's 32-bit parameters: {card}, budget {budget}")
        sys.exit(1)
    return {
        "workload": "N=8192 L=4 h=8 PBH lambda=32 (lambda_bar=21, ell=27) n=2^20 m=1024 planted=256 mu=526",
        "ms_per_query": round(1e3 * t, 3),
        "value": round(n * 526 / t, 1),
        "unit": "slot-comparisons/s",
        "offline_s": round(prep, 3),
        "paper_online_s": 0.83,
        "check": {"cardinality": card, "noise_budget_bits": budget},
    }


def batched_leg(pk, params, server, server_items, cfg, nq, steps, seed, plain_value, ab=True):
    """Config 'batched': nq queries, m log-uniform in [64, 2048], 25% planted, evaluated together
    under the library's schedule for nq queries (the whole call one captured HIP graph, replayed).
    Also: the same batch with eager launches (the graph's A/B), and with the select-and-sum on the
    vector units instead of the int8 matrix cores."""
    import torch
    import workload as W
    n, L = params.n, params.L
    g = W.rng(seed, "batch-sizes")
    sizes = np.rint(np.exp(g.uniform(np.log(64), np.log(2048), size=nq))).astype(int)
    log(f"[bench] batched leg: {nq} queries, m in [{sizes.min()}, {sizes.max()}]")
    qs = [make_query(params, server_items, cfg, int(m), int(round(0.25 * m)), seed + 100 * (i + 1))
          for i, m in enumerate(sizes)]
    outs = [torch.zeros((2, L, n), dtype=torch.int64, device="cuda") for _ in qs]
    args = ([q["cts"] for q in qs], [q["rlk"] for q in qs], [q["mask"] for q in qs], outs)

    def timed(k):
        server.eval_batch(*args)                  # warm-up (workspace, graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            server.eval_batch(*args)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k

    sched = server.schedule(nq).as_dict()
    t = timed(steps)
    bad = 0
    for q, o in zip(qs, outs):
        slots = torch.zeros((1, n), dtype=torch.int32, device="cuda")
        params.decrypt(q["sk"], o.reshape(1, 2, L, n), slots)
        torch.cuda.synchronize()
        card = int(slots.cpu().numpy().view(np.uint32).astype(np.int64).sum() % 65537)
        bad += card != q["planted"]
    if bad:
        log(f"[bench] WRONG RESULT in {bad} batched queries")
        sys.exit(1)
    ref = [o.clone() for o in outs]
    # event-timed eager run: the select-and-sum share
    server.timing(enable=True, reset=True)
    server.eval_batch(*args)
    tm = server.timing(enable=False)
    # A/B: eager launches; one select-and-sum launch per tile instead of per run; the select-and-sum
    # on the vector units
    t_eager = t_tiles = valu = None
    if ab:
        server.set_schedule(graph=pk.GRAPH_OFF)
        t_eager = timed(1)
    if ab and sched.get("run") == "one select-and-sum launch per run of tiles":
        server.set_schedule(run=pk.RUN_OFF)
        t_tiles = timed(1)
    if ab and server.plane_groups > 0:
        server.set_schedule(select_kernel=pk.SELECT_VALU)
        vs = server.schedule(nq).as_dict()
        t_valu = timed(1)
        valu = {"ms_per_query": round(1e3 * t_valu / nq, 3), "value": round(nq * n * cfg["mu"] / t_valu, 1),
                "speedup_vs_plain": round(nq * n * cfg["mu"] / t_valu / plain_value, 3),
                "schedule": vs}
    server.set_schedule(reset=True)
    if not all(torch.equal(a, b) for a, b in zip(ref, outs)):
        log("[bench] batched results differ between schedules")
        sys.exit(1)
    value = nq * n * cfg["mu"] / t
    roof = None
    if sched["select_kernel"].startswith("int8 matrix") and tm.select_sum_launches and tm.select_sum_ms > 0:
        # int8 multiply-adds of the digit-plane contraction: per computed batch, query, component,
        # limb and slot, ell code positions x 7 x 7 digit pairs, 2 operations each
        ops = server.max_load * nq * 2 * L * n * params.ell * MFMA_DIGIT_PAIRS * 2
        achieved = ops / (tm.select_sum_ms / 1e3)
        measured = pk.probe_mfma_int8()
        run_mode = sched.get("run") == "one select-and-sum launch per run of tiles"
        roof = {"kernel": "k_select_sum_planes_run" if run_mode else "k_select_sum_planes",
                "bound": "mfma", "achieved": round(achieved / 1e12, 1), "peak": INT8_DENSE_PEAK_T,
                "unit": "TOP/s (int8)", "frac": round(achieved / 1e12 / INT8_DENSE_PEAK_T, 4),
                "measured_instruction_peak": round(measured / 1e12, 1),
                "frac_of_measured": round(achieved / measured, 4),
                "launches": int(tm.select_sum_launches), "avg_launch_ms": round(tm.select_sum_ms / tm.select_sum_launches, 3),
                "ops_per_launch": int(ops / tm.select_sum_launches)}
    return {
        "queries": nq,
        "m_range": [int(sizes.min()), int(sizes.max())],
        "value": round(value, 1),
        "unit": "slot-comparisons/s",
        "ms_per_batch": round(1e3 * t, 2),
        "ms_per_query": round(1e3 * t / nq, 3),
        "speedup_vs_plain": round(value / plain_value, 3),
        "schedule": sched,
        "eager_ms_per_query": None if t_eager is None else round(1e3 * t_eager / nq, 3),
        "per_tile_select_sum_ms_per_query": None if t_tiles is None else round(1e3 * t_tiles / nq, 3),
        "select_sum_ms_per_batch": round(tm.select_sum_ms, 2),
        "checked_cardinalities": nq,
        "batches_computed": int(server.max_load),
        "value_computed_batches": round(nq * n * server.max_load / t, 1),
        "valu_select_sum": valu,
        "roofline_mfma": roof,
    }


def large_leg(pk, steps, nq, seed):
    """The large configuration (N = 16384, L = 8, h = 4, ell = 569, n = 2^24 32-bit items, m = 4096
    with 1024 planted, mu = 3487): the plaintexts (2.1 TB) are not resident, so every query
    regenerates them per tile; plain single queries, then one batch of nq queries sharing the
    generation (m log-uniform in [1024, 4096], 25% planted)."""
    import torch
    import workload as W
    cfg = CONFIGS["large"]
    n, L = 1 << cfg["log_n"], cfg["L"]
    params = pk.Params(cfg["log_n"], L, cfg["h"], cfg["item_bits"], cfg["mu"])
    items = W.server_items(cfg["n_server"], cfg["item_bits"], seed)
    t0 = time.perf_counter()
    server = pk.Server(params, items, cache_plaintexts=False)
    torch.cuda.synchronize()
    prep = time.perf_counter() - t0
    log(f"[bench] large leg: server ready in {prep:.1f} s, max load {server.max_load}")
    q = make_query(params, items, cfg, cfg["m_client"], cfg["planted"], seed + 1)
    out = torch.zeros((2, L, n), dtype=torch.int64, device="cuda")
    server.eval(q["cts"], q["rlk"], q["mask"], out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        server.eval(q["cts"], q["rlk"], q["mask"], out)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / steps
    slots = torch.zeros((1, n), dtype=torch.int32, device="cuda")
    params.decrypt(q["sk"], out.reshape(1, 2, L, n), slots)
    torch.cuda.synchronize()
    card = int(slots.cpu().numpy().view(np.uint32).astype(np.int64).sum() % 65537)
    budget = params.noise_budget(q["sk"], out)
    if card != cfg["planted"] or budget <= 0:
        log(f"[bench] WRONG RESULT in the large leg: {card}, budget {budget}")
        sys.exit(1)
    g = W.rng(seed, "large-batch-sizes")
    sizes = np.rint(np.exp(g.uniform(np.log(1024), np.log(4096), size=nq))).astype(int)
    qs = [q] + [make_query(params, items, cfg, int(m), int(round(0.25 * m)), seed + 100 * (i + 2))
                for i, m in enumerate(sizes[1:])]
    outs = [torch.zeros((2, L, n), dtype=torch.int64, device="cuda") for _ in qs]
    args = ([x["cts"] for x in qs], [x["rlk"] for x in qs], [x["mask"] for x in qs], outs)
    server.eval_batch(*args)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    server.eval_batch(*args)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    bad = int(not torch.equal(outs[0], out))
    for x, o in zip(qs[1:], outs[1:]):
        params.decrypt(x["sk"], o.reshape(1, 2, L, n), slots)
        torch.cuda.synchronize()
        bad += int(slots.cpu().numpy().view(np.uint32).astype(np.int64).sum() % 65537) != x["planted"]
    if bad:
        log(f"[bench] WRONG RESULT in {bad} batched queries of the large leg")
        sys.exit(1)
    max_load = int(server.max_load)
    server.close()
    v_plain = n * cfg["mu"] / t_plain
    v_batch = nq * n * cfg["mu"] / t_batch
    return {
        "workload": (f"large: N={n} L={L} t=65537 h={cfg['h']} ell={params.ell} b={n} mu={cfg['mu']} "
                     f"n={cfg['n_server']} m={cfg['m_client']} planted={cfg['planted']}, plaintexts generated "
                     f"per tile"),
        "offline_s": round(prep, 2),
        "batches_computed": max_load,
        "plain": {"ms_per_query": round(1e3 * t_plain, 1), "value": round(v_plain, 1),
                  "unit": "slot-comparisons/s", "steps": steps,
                  "check": {"cardinality": card, "noise_budget_bits": budget}},
        "batched": {"queries": nq, "m_range": [int(min(cfg["m_client"], sizes[1:].min(initial=4096))),
                                               int(max(cfg["m_client"], sizes[1:].max(initial=0)))],
                    "ms_per_query": round(1e3 * t_batch / nq, 1), "value": round(v_batch, 1),
                    "unit": "slot-comparisons/s", "speedup_vs_plain": round(v_batch / v_plain, 3),
                    "checked": "first query equals its single-query result; every cardinality"},
    }


# Large elements (Table "psisum-eval": PSI-Sum, b = 16384, n = 2^20, mu = 296, m = 1024): 32-byte
# strings hashed to lambda = 40 + ceil(log2(b mu)) = 63 bits, permutation-based hashing (stored
# values of 51 bits with the hash index), h = 16 (N = 2^14 from Table "mod-per-hamming-weight"),
# 5 primes (270 bits against the table's 240), 12-bit server values.
LARGE_ELEMENTS = dict(log_n=14, L=5, h=16, mu=296, n_server=1 << 20, m_client=1024, planted=256, length=32)


def large_elements_leg(pk, steps, seed):
    """PSI-Sum over large elements at the shape of Table "psisum-eval" (n = 2^20)."""
    import torch
    import workload as W
    c = LARGE_ELEMENTS
    n, L = 1 << c["log_n"], c["L"]
    lam = pk.large_element_bits(n, 1, c["mu"])
    params = pk.Params(c["log_n"], L, c["h"], lam, c["mu"], pbh=True)
    server_e = W.byte_elements(c["n_server"], c["length"], seed)
    t0 = time.perf_counter()
    hs = pk.hash_elements(server_e, lam)
    t_hash = time.perf_counter() - t0
    values = W.item_values(c["n_server"], 0, 1 << 12, seed + 1)
    t0 = time.perf_counter()
    server = pk.Server(params, hs, cache_plaintexts=True, values=values)
    torch.cuda.synchronize()
    prep = time.perf_counter() - t0
    g = W.rng(seed, "large-elements-client")
    common = np.sort(g.choice(c["n_server"], size=c["planted"], replace=False))
    fresh = W.byte_elements(c["m_client"] - c["planted"], c["length"], seed + 2, tag="client-elements")
    client_e = np.concatenate([server_e[common], fresh])[g.permutation(c["m_client"])]
    hc = pk.hash_elements(client_e, lam)
    table, valid = params.client_table(hc)
    planes = params.codeword_planes(table, valid)
    ell = params.ell
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed + 3)
    sk = dev(W.secret_key(n, seed + 4))
    a = torch.stack([torch.randint(0, q, (ell, n), generator=gen, device="cuda", dtype=torch.int64)
                     for q in params.q_primes], dim=1).contiguous()
    e = torch.clamp(torch.round(torch.randn((ell, n), generator=gen, device="cuda") * 3.2), -19, 19).to(torch.int32)
    cts = torch.empty((ell, 2, L, n), dtype=torch.int64, device="cuda")
    params.encrypt(sk, dev(planes), a, e, cts)
    ka = torch.stack([torch.randint(0, q, (L, n), generator=gen, device="cuda", dtype=torch.int64)
                      for q in params.q_primes], dim=1).contiguous()
    ke = torch.clamp(torch.round(torch.randn((L, n), generator=gen, device="cuda") * 3.2), -19, 19).to(torch.int32)
    rlk = torch.empty((L, 2, L, n), dtype=torch.int64, device="cuda")
    params.keygen_relin(sk, ka, ke, rlk)
    mask = dev(W.zero_sum_mask(n, 65537, seed + 5))
    out = torch.zeros((2, L, n), dtype=torch.int64, device="cuda")
    server.eval(cts, rlk, mask, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        server.eval(cts, rlk, mask, out)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / steps
    slots = torch.zeros((1, n), dtype=torch.int32, device="cuda")
    params.decrypt(sk, out.reshape(1, 2, L, n), slots)
    torch.cuda.synchronize()
    got = int(slots.cpu().numpy().view(np.uint32).astype(np.int64).sum() % 65537)
    want = int(values[common].astype(np.int64).sum() % 65537)
    budget = params.noise_budget(sk, out)
    max_load = int(server.max_load)
    server.close()
    if got != want or budget <= 0:
        log(f"[bench] WRONG PSI-Sum over large elements: {got} (want {want}), budget {budget}")
        sys.exit(1)
    return {
        "workload": (f"PSI-Sum over {c['length']}-byte elements: N=b={n} L={L} h={c['h']} lambda={lam} "
                     f"(PBH, stored {params.effective_bits} bits) ell={ell} n=2^20 mu={c['mu']} m={c['m_client']} "
                     f"planted={c['planted']}, 12-bit values, plaintexts cached"),
        "ms_per_query": round(1e3 * t, 3),
        "value": round(n * c["mu"] / t, 1),
        "unit": "slot-comparisons/s",
        "steps": steps,
        "batches_computed": max_load,
        "hash_s": round(t_hash, 3),
        "offline_s": round(prep, 3),
        "paper_online_s": 7.0,
        "check": {"sum_mod_t": got, "noise_budget_bits": budget},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", choices=sorted(CONFIGS), default="paper")
    ap.add_argument("--mode", choices=["cached", "generate"], default="cached",
                    help="server plaintexts resident in NTT form (cached) or regenerated each query")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=64, help="queries per batched launch (0: skip the batched leg)")
    ap.add_argument("--batch-steps", type=int, default=2)
    ap.add_argument("--no-batch-ab", action="store_true",
                    help="batched leg: only the library's schedule (no eager, per-tile or vector-unit A/B runs)")
    ap.add_argument("--seed", type=int, default=2024)
    ap.add_argument("--psi-sum-steps", type=int, default=5, help="steps of the PSI-Sum leg (0: skip it)")
    ap.add_argument("--paper32-steps", type=int, default=5,
                    help="steps of the leg with the paper's own 32-bit parameters (0: skip it)")
    ap.add_argument("--large-steps", type=int, default=2,
                    help="single queries timed in the large-configuration leg (0: skip the leg)")
    ap.add_argument("--large-batch", type=int, default=4, help="queries of the large leg's batch")
    ap.add_argument("--large-elements-steps", type=int, default=3,
                    help="steps of the PSI-Sum leg over large (hashed 32-byte) elements (0: skip it)")
    ap.add_argument("--serve", type=int, default=500, help="requests in the serving leg (0: skip it)")
    ap.add_argument("--serve-pool", type=int, default=16, help="distinct client queries behind the requests")
    ap.add_argument("--serve-slots", type=int, default=0,
                    help="maximum query slots of the serving leg (0: as many as its HBM budget admits)")
    ap.add_argument("--serve-store", choices=["cache", "planes"], default="planes",
                    help="serving server keeps the NTT-form cache, or only int8 digit planes")
    ap.add_argument("--serve-load", type=float, default=0.8, help="arrival rate / saturated capacity")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the plain leg, run one elementwise negation of MIB MiB of int64 (a copy kernel "
                         "of known traffic, for scaling hardware byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only; sharding the server computation over several GPUs "
              "is described in the design notes, not measured", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2310_14565_amd as pk
    import workload as W

    cfg = CONFIGS[args.config]
    n = 1 << cfg["log_n"]
    L = cfg["L"]
    torch.cuda.set_device(0)
    log(f"[bench] config={args.config} mode={args.mode} N={n} L={L} h={cfg['h']} mu={cfg['mu']}")
    params = pk.Params(cfg["log_n"], L, cfg["h"], cfg["item_bits"], cfg["mu"])
    ell = params.ell
    server_items = W.server_items(cfg["n_server"], cfg["item_bits"], args.seed)
    client_items = W.client_items(cfg["m_client"], server_items, cfg["planted"], cfg["item_bits"], args.seed + 1)

    # client request (GPU encryption of the codeword bit planes) and keys
    table, valid = params.client_table(client_items)
    planes = params.codeword_planes(table, valid)
    sk = dev(W.secret_key(n, args.seed + 2))
    cts = torch.zeros((ell, 2, L, n), dtype=torch.int64, device="cuda")
    chunk = 64
    for j0 in range(0, ell, chunk):
        j1 = min(ell, j0 + chunk)
        a = W.uniform_residues((j1 - j0,), params.q_primes, n, args.seed + 3 + j0, "enc-a")
        e = W.errors((j1 - j0, n), args.seed + 3 + j0, "enc-e")
        params.encrypt(sk, dev(planes[j0:j1]), dev(a), dev(e), cts[j0:j1])
    rlk = torch.zeros((L, 2, L, n), dtype=torch.int64, device="cuda")
    params.keygen_relin(sk, dev(W.uniform_residues((L,), params.q_primes, n, args.seed + 4, "rlk-a")),
                        dev(W.errors((L, n), args.seed + 4, "rlk-e")), rlk)
    mask = dev(W.zero_sum_mask(n, 65537, args.seed + 5))
    torch.cuda.synchronize()

    log("[bench] server preparation")
    t0 = time.perf_counter()
    server = pk.Server(params, server_items, cache_plaintexts=(args.mode == "cached"))
    torch.cuda.synchronize()
    offline_s = time.perf_counter() - t0
    log(f"[bench] offline {offline_s:.2f} s, max load {server.max_load}, cached={server.cached}")

    out = torch.zeros((2, L, n), dtype=torch.int64, device="cuda")
    for _ in range(args.warmup):
        server.eval(cts, rlk, mask, out)
    torch.cuda.synchronize()
    log("[bench] warmup done")

    server.timing(enable=True, reset=True)
    per_step = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        s0 = time.perf_counter()
        server.eval(cts, rlk, mask, out)
        torch.cuda.synchronize()
        per_step.append(time.perf_counter() - s0)
    t_total = time.perf_counter() - t_start
    tm = server.timing(enable=False)
    log(f"[bench] timed {args.steps} steps in {t_total:.3f} s")

    # the result of the last step must decrypt to the planted cardinality
    slots = torch.zeros((1, n), dtype=torch.int32, device="cuda")
    params.decrypt(sk, out.reshape(1, 2, L, n), slots)
    torch.cuda.synchronize()
    card = int(slots.cpu().numpy().view(np.uint32).astype(np.int64).sum() % 65537)
    budget = params.noise_budget(sk, out)
    if card != cfg["planted"] or budget <= 0:
        log(f"[bench] WRONG RESULT: cardinality {card} (want {cfg['planted']}), noise budget {budget}")
        sys.exit(1)

    ms_per_step = 1e3 * t_total / args.steps
    comparisons = n * cfg["mu"]
    value = comparisons * args.steps / t_total
    launches = max(tm.select_sum_launches, 1)
    avg_ms = tm.select_sum_ms / launches
    bytes_per_launch = tm.select_sum_bytes / launches
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9 if avg_ms > 0 else 0.0
    # the committed byte counts were taken on the paper-shaped workload with resident plaintexts
    trec = traffic_record("select_sum") if (args.config == "paper" and args.mode == "cached") else None
    roofline = {
        "bound": "hbm",
        "kernel": "k_select_sum",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None if trec is None else trec["bytes_per_launch"],
        "launches_per_step": tm.select_sum_launches / args.steps,
        "avg_launch_ms": round(avg_ms, 4),
        "algorithmic_bytes_per_launch": int(bytes_per_launch),
        "select_sum_ms_per_step": round(tm.select_sum_ms / args.steps, 3),
        "eval_event_ms_per_step": round(tm.eval_ms / max(tm.evals, 1), 3),
    }
    line = {
        "metric": ("server item-comparisons/sec at m=1024,n=2^20 (plain one-query-per-launch path)"
                   if args.config == "paper" else
                   f"server item-comparisons/sec at m={cfg['m_client']},n={cfg['n_server']} (plain path)"),
        "value": round(value, 1),
        "unit": "slot-comparisons/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (seeded random 32-bit sets, planted intersection)",
        "config": {
            "workload": (f"{args.config}: N={n} L={L} t=65537 h={cfg['h']} ell={ell} b={n} mu={cfg['mu']} "
                         f"n={cfg['n_server']} m={cfg['m_client']} planted={cfg['planted']}, "
                         f"server plaintexts {args.mode}"),
            "path": "plain",
            "global_batch": 1,
        },
        "roofline": roofline,
        "latency_ms": {"p50": round(1e3 * float(np.percentile(per_step, 50)), 3),
                       "p99": round(1e3 * float(np.percentile(per_step, 99)), 3)},
        "offline_s": round(offline_s, 3),
        "server_max_load": server.max_load,
        "batches_computed": int(server.max_load),
        "value_computed_batches": round(n * server.max_load * args.steps / t_total, 1),
        "value_note": ("value counts b * mu slot comparisons per query; batches at or above the fullest bin hold "
                       "only dummies, their equality ciphertext is exactly zero and they are skipped, so "
                       "value_computed_batches counts only the batches the kernels run"),
        "check": {"cardinality": card, "noise_budget_bits": budget},
    }
    line["roofline_valu"] = valu_roofline(pk, tm, n)
    line["compression"] = compression_leg(params, out, args.seed + 17)
    if args.copy_calibration > 0:
        words = (args.copy_calibration << 20) // 8
        src = torch.ones(words, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        line["copy_calibration_bytes"] = {"read": words * 8, "written": words * 8}
        del src, dst
    if args.batch > 0:
        line["batched"] = batched_leg(pk, params, server, server_items, cfg, args.batch, args.batch_steps,
                                      args.seed + 7, value, ab=not args.no_batch_ab)
    if args.psi_sum_steps > 0 and args.config == "paper":
        server.close()
        line["psi_sum"] = psi_sum_leg(pk, params, server_items, cfg, args.psi_sum_steps, args.seed + 9)
    if args.paper32_steps > 0 and args.config == "paper":
        server.close()
        line["paper32"] = paper32_leg(pk, args.paper32_steps, args.seed + 13)
    if args.large_elements_steps > 0 and args.config == "paper":
        server.close()
        torch.cuda.empty_cache()
        line["large_elements"] = large_elements_leg(pk, args.large_elements_steps, args.seed + 23)
    if args.large_steps > 0 and args.config == "paper":
        server.close()
        torch.cuda.empty_cache()
        line["large"] = large_leg(pk, args.large_steps, args.large_batch, args.seed + 19)
    if args.serve > 0:
        server.close()
        del cts, rlk, out
        torch.cuda.empty_cache()
        line["serving"] = serving_leg(pk, args.serve, args.serve_pool, args.serve_slots, args.serve_load,
                                      args.seed + 11, planes_only=args.serve_store == "planes")
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle sample)")
        line["cpu_baseline"] = cpu_baseline(cfg, params, server_items, args.seed, line["batches_computed"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
