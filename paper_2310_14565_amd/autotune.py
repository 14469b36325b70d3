"""Autotuner of the batched server computation's schedule (pepsi_schedule).

For each workload (parameter set, server set and number of queries) it times every candidate
schedule -- tile of 16, 32 or 64 server batches, the int8 matrix-core or the 64-bit VALU
select-and-sum, a captured HIP graph or eager launches -- on the current GPU and writes the
fastest into csrc/schedule_table.inc, which the library compiles in (rebuild after running).
Each entry keeps every candidate's time as a comment.  Requests are seeded uniform
ciphertexts: the kernels' work does not depend on the values.

    python -m paper_2310_14565_amd.autotune [--quick] [--out FILE]
"""
from __future__ import annotations

import argparse
import itertools
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
TABLE = os.path.join(HERE, "csrc", "schedule_table.inc")

# (name, log_n, L, h, item_bits, mu, n_server, query counts)
WORKLOADS = [
    ("paper-shaped", 13, 4, 4, 32, 526, 1 << 20, (8, 16, 32, 64)),
]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def tune(pk, name, log_n, L, h, bits, mu, n_server, counts, reps):
    import torch
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import workload as W
    n = 1 << log_n
    params = pk.Params(log_n, L, h, bits, mu)
    server = pk.Server(params, W.server_items(n_server, bits, 2024), cache_plaintexts=True)
    log(f"[autotune] {name}: ell={params.ell} max_load={server.max_load} planes={server.plane_groups}")
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    nmax = max(counts)
    qp = torch.tensor(params.q_primes, dtype=torch.int64, device="cuda")

    def residues(*shape):
        x = torch.randint(0, 1 << 62, shape + (L, n), generator=g, device="cuda", dtype=torch.int64)
        return (x % qp[:, None]).contiguous()

    cts = [residues(params.ell, 2) for _ in range(nmax)]
    rlk = [residues(L, 2) for _ in range(nmax)]
    outs = [torch.zeros((2, L, n), dtype=torch.int64, device="cuda") for _ in range(nmax)]
    kernels = [pk.SELECT_PLANES, pk.SELECT_VALU] if server.plane_groups > 0 else [pk.SELECT_VALU]
    entries = []
    for nq in sorted(counts):
        times = {}
        cands = [(t, k, g, r) for t, k, g, r in itertools.product((16, 32, 64), kernels, (pk.GRAPH_ON, pk.GRAPH_OFF),
                                                                  (pk.RUN_ON, pk.RUN_OFF))
                 if k == pk.SELECT_PLANES or r == pk.RUN_OFF]
        for tile, kern, graph, run in cands:
            server.set_schedule(tile_batches=tile, select_kernel=kern, graph=graph, run=run)
            args = (cts[:nq], rlk[:nq], None, outs[:nq])
            try:
                server.eval_batch(*args)                     # sets the workspace up (and captures)
                torch.cuda.synchronize()
            except pk.PepsiError as e:
                log(f"[autotune]   nq={nq} tile={tile} kernel={kern} graph={graph} run={run}: {e}")
                continue
            t0 = time.perf_counter()
            for _ in range(reps):
                server.eval_batch(*args)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0) / reps / nq
            times[(tile, kern, graph, run)] = ms
            log(f"[autotune]   nq={nq} tile={tile} kernel={kern} graph={graph} run={run}: {ms:.3f} ms/query")
        server.set_schedule(reset=True)
        best = choose(times)
        entries.append((log_n, L, params.ell, h, nq, best, times[best], times))
    server.close()
    del cts, rlk, outs
    torch.cuda.empty_cache()
    return entries


def choose(times: dict):
    """The fastest candidate; among those within TIE of it (run-to-run noise), the captured graph
    first, then the larger tile."""
    best = min(times.values())
    near = [c for c, v in times.items() if v <= best * (1 + TIE)]
    return min(near, key=lambda c: (c[2] != 1, -c[0], times[c]))


def _key(c) -> str:
    t, k, g, r = c
    return f"{t}/{NAMES[k]}/{'g' if g == 1 else 'e'}/{'run' if r == 1 else 'tile'}"


TIE = 0.005
NAMES = {1: "planes", 2: "valu"}


def parse_table(path):
    """Entries of a written table, from its candidate comments (for --rewrite)."""
    import re
    entries, pending = [], None
    for line in open(path):
        m = re.match(r"// nq <= (\d+): (.*)", line)
        if m:
            times = {}
            for item in m.group(2).split(", "):
                key, v = item.split(": ")
                parts = key.split("/")
                t, k, g = parts[:3]
                r = 1 if len(parts) > 3 and parts[3] == "run" else 2      # tables before run mode: per tile
                times[(int(t), {"planes": 1, "valu": 2}[k], 1 if g == "g" else 2, r)] = float(v)
            pending = (int(m.group(1)), times)
            continue
        m = re.match(r"\{(\d+), (\d+), (\d+), (\d+), (\d+),", line)
        if m and pending:
            log_n, L, ell, h, nq = map(int, m.groups())
            times = pending[1]
            best = choose(times)
            entries.append((log_n, L, ell, h, nq, best, times[best], times))
            pending = None
    return entries


def write_table(entries, path, device):
    names = NAMES
    lines = ["// Written by paper_2310_14565_amd/autotune.py on " + device + ".",
             "// {log_n, L, ell, h, nq_max, tile_batches, select_kernel (1 planes, 2 VALU), graph (1 on, 2 off),",
             "//  run (1 one select-and-sum launch per run of tiles, 2 one per tile), ms per query}; the comment",
             "//  lists every candidate as tile/kernel/graph/run: ms per query."]
    for (log_n, L, ell, h, nq, (tile, kern, graph, run), ms, times) in entries:
        cands = ", ".join(f"{_key(c)}: {v:.3f}" for c, v in sorted(times.items()))
        lines.append(f"// nq <= {nq}: {cands}")
        lines.append(f"{{{log_n}, {L}, {ell}, {h}, {nq}, {tile}, {kern}, {graph}, {run}, {ms:.3f}}},")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--quick", action="store_true", help="only the largest query count of each workload")
    ap.add_argument("--rewrite", metavar="TABLE",
                    help="no measurement: re-choose the entries of a written table from its candidate times")
    ap.add_argument("--device", default="MI355X", help="device name written with --rewrite")
    args = ap.parse_args()
    if args.rewrite:
        write_table(parse_table(args.rewrite), args.out, args.device)
        log(f"[autotune] rewrote {args.out} from {args.rewrite}")
        return
    import torch
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import paper_2310_14565_amd as pk
    torch.cuda.set_device(0)
    entries = []
    for name, log_n, L, h, bits, mu, n_server, counts in WORKLOADS:
        if args.quick:
            counts = (max(counts),)
        entries += tune(pk, name, log_n, L, h, bits, mu, n_server, counts, args.reps)
    write_table(entries, args.out, torch.cuda.get_device_name(0))
    log(f"[autotune] wrote {len(entries)} entries to {args.out}")


if __name__ == "__main__":
    main()
