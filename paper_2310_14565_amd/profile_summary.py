"""Summaries of rocprofv3 databases of bench.py runs (the text kept under profiles/).

    python paper_2310_14565_amd/profile_summary.py kernels KT.db
        per-kernel time per evaluation of the plain path (from the first k_select_sum to the
        VALU probes, per k_select_sum launch) and of the batched path (from there to the
        matrix-instruction probe or the vector-unit A/B, per query), from a --kernel-trace
        database;
    python paper_2310_14565_amd/profile_summary.py counters PMC.db
        per-kernel VALU issue (VALUBusy = SQ_ACTIVE_INST_VALU / CUs / per-XCD GRBM_GUI_ACTIVE),
        VALU instructions, LDS bank conflicts per LDS instruction, from a --pmc database;
    python paper_2310_14565_amd/profile_summary.py totals PMC.db
        every counter summed per kernel, with the matrix pipe's busy share and the waves' wait
        shares where those counters were taken;
    python paper_2310_14565_amd/profile_summary.py traffic FETCH.db WRITE.db BENCH.json
        per-kernel HBM bytes per dispatch from FETCH_SIZE and WRITE_SIZE (KiB), each scaled by
        what the counter reads for the copy kernel of bench.py --copy-calibration (torch.neg of
        a known size; its read and written bytes come from the bench line, BENCH.json).
"""
from __future__ import annotations

import collections
import json
import re
import sqlite3
import sys

CU = 256
XCD = 8


def short(name: str) -> str:
    n = name.replace("pepsi::(anonymous namespace)::", "").replace("(pepsi::NttLoad)", "L")
    n = n.replace("(pepsi::NttStore)", "S").replace("(pepsi::InvProducts)", "I")
    n = re.sub(r"^void ", "", n)
    n = re.sub(r"\(Tables.*|\(unsigned.*|\(long.*", "", n)
    return n[:64]


def kernels(db_path: str):
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, start, end from kernels order by start").fetchall()
    names = [short(r[0]) for r in rows]

    def first(pred, start=0):
        for i in range(start, len(rows)):
            if pred(names[i]):
                return i
        return len(rows)

    def window(a, b, label, unit):
        agg = collections.OrderedDict()
        for i in range(a, b):
            c, t = agg.get(names[i], (0, 0.0))
            agg[names[i]] = (c + 1, t + (rows[i][2] - rows[i][1]) / 1e6)
        div = agg.get(unit, (0, 0))[0]
        if not div:
            return
        tot = sum(t for _, t in agg.values())
        print(f"== {label}: {b - a} dispatches, {div} evaluations ({unit} launches), "
              f"{tot / div:.3f} ms of kernels per evaluation")
        print(f"  {'ms/eval':>9s} {'share':>6s} {'calls/eval':>10s} {'avg us':>10s}  kernel")
        for n, (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
            if t / tot < 0.001:
                continue
            print(f"  {t / div:9.4f} {100 * t / tot:5.1f}% {c / div:10.2f} {1e3 * t / c:10.2f}  {n}")

    # bench.py order: plain evaluations (one k_select_sum each), the VALU probes, then the batched
    # leg (one k_request_planes per query), then its matrix-instruction probe and its
    # vector-unit A/B (k_select_sum_multi); the batched window ends at whichever comes first
    a = first(lambda n: n == "k_select_sum")
    p = first(lambda n: "probe" in n, a)
    window(a, p, "plain path", "k_select_sum")
    b0 = first(lambda n: "k_request_planes" in n, p)
    bm = first(lambda n: "k_select_sum_multi" in n or "probe" in n, b0)
    window(b0, bm, "batched path", "k_request_planes")


def counters(db_path: str):
    db = sqlite3.connect(db_path)
    rows = db.execute("select dispatch_id, kernel_name, counter_name, value, duration from counters_collection").fetchall()
    disp = collections.defaultdict(dict)
    meta = {}
    for d, k, c, v, dur in rows:
        disp[d][c] = disp[d].get(c, 0.0) + v
        meta[d] = (short(k), dur)
    order = sorted(disp)
    # the plain path from its first k_select_sum (server preparation before it is left out), the
    # batched leg from its first k_request_planes (one per query)
    start = next((d for d in order if meta[d][0] == "k_select_sum"), order[0])
    split = next((d for d in order if meta[d][0] == "k_request_planes"), None)
    for label, ids in (("plain path", [d for d in order if start <= d and (split is None or d < split)]),
                       ("batched path", [d for d in order if split is not None and d >= split])):
        if not ids:
            continue
        agg = collections.defaultdict(lambda: collections.defaultdict(float))
        for d in ids:
            k, dur = meta[d]
            agg[k]["n"] += 1
            agg[k]["dur"] += dur
            for c, v in disp[d].items():
                agg[k][c] += v
        tot = sum(a["dur"] for a in agg.values())
        print(f"== {label}: {len(ids)} dispatches")
        print(f"  {'kernel':46s} {'calls':>5s} {'ms':>8s} {'VALUBusy%':>9s} {'VALU inst/wave':>14s} "
              f"{'SALU/VALU':>9s} {'LDS conf/inst':>13s}")
        for k, a in sorted(agg.items(), key=lambda kv: -kv[1]["dur"]):
            if a["dur"] < 0.005 * tot:
                continue
            grbm = a.get("GRBM_GUI_ACTIVE", 0) / XCD
            busy = 100 * a.get("SQ_ACTIVE_INST_VALU", 0) / CU / grbm if grbm else 0
            lds = a.get("SQ_ACTIVE_INST_LDS", 0)
            conf = a.get("SQ_LDS_BANK_CONFLICT", 0) / lds if lds else 0
            waves = a.get("SQ_WAVES", 0)
            valu = a.get("SQ_INSTS_VALU", 0)
            print(f"  {k:46s} {int(a['n']):5d} {a['dur'] / 1e6:8.2f} {busy:9.1f} "
                  f"{valu / waves if waves else 0:14.0f} {a.get('SQ_INSTS_SALU', 0) / valu if valu else 0:9.3f} "
                  f"{conf:13.3f}")


def traffic(fetch_db: str, write_db: str, calib_json: str | None):
    def per_kernel(db_path, counter):
        db = sqlite3.connect(db_path)
        rows = db.execute("select dispatch_id, kernel_name, value from counters_collection where counter_name = ?",
                          (counter,)).fetchall()
        disp = collections.defaultdict(float)
        meta = {}
        for d, k, v in rows:
            disp[d] += v
            meta[d] = k
        agg = collections.defaultdict(list)
        for d in sorted(disp):
            agg[meta[d]].append(disp[d] * 1024.0)          # KiB -> bytes
        return agg

    f = per_kernel(fetch_db, "FETCH_SIZE")
    w = per_kernel(write_db, "WRITE_SIZE")
    neg = [k for k in f if "neg_kernel" in k]
    fs = ws = 1.0
    if neg and calib_json:
        line = [json.loads(x) for x in open(calib_json) if x.startswith("{")][-1]
        cal = line.get("copy_calibration_bytes", {})
        fs = cal["read"] / max(f[neg[0]])
        ws = cal["written"] / max(w.get(neg[0], [1.0]))
        print(f"copy calibration ({short(neg[0])}, {cal['read'] / 2**30:.1f} GiB read and written): "
              f"{fs:.4f} bytes read per counted FETCH_SIZE byte, {ws:.4f} written per counted WRITE_SIZE byte")
    print(f"  {'kernel':46s} {'disp':>5s} {'read GB/disp':>12s} {'written GB/disp':>15s}")
    for k in sorted(f, key=lambda k: -sum(f[k])):
        if k in neg:
            continue
        fk, wk = f[k], w.get(k, [0.0])
        print(f"  {short(k):46s} {len(fk):5d} {fs * sum(fk) / len(fk) / 1e9:12.3f} "
              f"{ws * sum(wk) / len(wk) / 1e9:15.3f}")
        if len(fk) <= 24:
            print("    per dispatch, read GB: " + " ".join(f"{fs * v / 1e9:.2f}" for v in fk))
            print("    per dispatch, written GB: " + " ".join(f"{ws * v / 1e9:.2f}" for v in wk))


def totals(db_path: str):
    """Every counter summed over each kernel's dispatches, with the matrix-pipe and wait shares."""
    db = sqlite3.connect(db_path)
    rows = db.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection").fetchall()
    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    for d, k, c, v in rows:
        agg[short(k)][c] += v
        disp[short(k)].add(d)
    for k, a in agg.items():
        print(f"== {k}: {len(disp[k])} dispatches")
        for c in sorted(a):
            print(f"  {c:28s} {a[c]:.6g}")
        grbm = a.get("GRBM_GUI_ACTIVE", 0) / XCD
        if grbm and "SQ_VALU_MFMA_BUSY_CYCLES" in a:
            print(f"  matrix pipe busy: {a['SQ_VALU_MFMA_BUSY_CYCLES'] / (4 * CU) / grbm:.3f} "
                  f"(SQ_VALU_MFMA_BUSY_CYCLES / 1024 SIMDs / (GRBM_GUI_ACTIVE / 8))")
        if a.get("SQ_WAVE_CYCLES"):
            for c in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY"):
                if c in a:
                    print(f"  {c} / SQ_WAVE_CYCLES: {a[c] / a['SQ_WAVE_CYCLES']:.3f}")
        if a.get("SQ_INSTS_MFMA") and a.get("SQ_INSTS_VALU"):
            print(f"  other VALU instructions per matrix instruction: "
                  f"{(a['SQ_INSTS_VALU'] - a['SQ_INSTS_MFMA']) / a['SQ_INSTS_MFMA']:.2f}")


def main():
    if len(sys.argv) < 3:
        print(__doc__)
        sys.exit(2)
    cmd = sys.argv[1]
    if cmd == "kernels":
        kernels(sys.argv[2])
    elif cmd == "counters":
        counters(sys.argv[2])
    elif cmd == "totals":
        totals(sys.argv[2])
    elif cmd == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4] if len(sys.argv) > 4 else None)
    else:
        print(__doc__)
        sys.exit(2)


if __name__ == "__main__":
    main()
