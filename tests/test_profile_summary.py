"""The rocprofv3 summary tool on small synthetic databases (same tables and columns as rocprofv3's
rocpd output: a `kernels` view and a `counters_collection` view)."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TOOL = os.path.join(ROOT, "paper_2310_14565_amd", "profile_summary.py")


def run(*args):
    r = subprocess.run([sys.executable, TOOL, *args], capture_output=True, text=True, check=True)
    return r.stdout


def kernel_db(path, names_us):
    db = sqlite3.connect(path)
    db.execute("create table kernels (name text, start integer, end integer)")
    t = 0
    for name, us in names_us:
        db.execute("insert into kernels values (?, ?, ?)", (name, t, t + int(us * 1000)))
        t += int(us * 1000) + 10
    db.commit()
    db.close()


def counter_db(path, rows):
    db = sqlite3.connect(path)
    db.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
               "value real, duration integer)")
    db.executemany("insert into counters_collection values (?, ?, ?, ?, ?)", rows)
    db.commit()
    db.close()


def test_kernels_windows_per_evaluation(tmp_path):
    seq = [("void pepsi::(anonymous namespace)::k_encode<13, 4>(Tables)", 5.0)]
    for _ in range(2):                                   # two plain evaluations
        seq += [("pepsi::(anonymous namespace)::k_select_sum(Tables, int)", 100.0),
                ("void pepsi::(anonymous namespace)::k_ntt_inv<13, 0, 3>(Tables)", 10.0)]
    seq += [("void pepsi::(anonymous namespace)::k_probe_valu<0>(unsigned)", 50.0)]
    for _ in range(4):                                   # four batched queries
        seq += [("pepsi::(anonymous namespace)::k_request_planes(Tables, int)", 2.0),
                ("void pepsi::(anonymous namespace)::k_ntt_inv<13, 0, 3>(Tables)", 4.0)]
    seq += [("void pepsi::(anonymous namespace)::k_probe_valu<6>(unsigned)", 30.0),
            ("pepsi::(anonymous namespace)::k_select_sum_multi(Tables, int)", 7.0)]
    db = str(tmp_path / "kt.db")
    kernel_db(db, seq)
    out = run("kernels", db)
    plain, batched = out.split("== batched path")
    assert "2 evaluations (k_select_sum launches), 0.110 ms" in plain
    assert "4 evaluations (k_request_planes launches), 0.006 ms" in batched
    assert "k_probe_valu" not in out and "k_select_sum_multi" not in out


def test_counters_busy_share_and_split(tmp_path):
    # one plain dispatch and one batched one; 8 XCDs x 1000 active cycles, 256 CUs x 500 VALU cycles
    rows = []
    for d, k in ((1, "k_select_sum"), (2, "k_request_planes")):
        for c, v in (("GRBM_GUI_ACTIVE", 8000.0), ("SQ_ACTIVE_INST_VALU", 256 * 500.0), ("SQ_INSTS_VALU", 640.0),
                     ("SQ_WAVES", 10.0), ("SQ_INSTS_SALU", 64.0), ("SQ_ACTIVE_INST_LDS", 4.0),
                     ("SQ_LDS_BANK_CONFLICT", 2.0)):
            rows.append((d, "pepsi::(anonymous namespace)::%s(Tables)" % k, c, v, 1000000))
    db = str(tmp_path / "c.db")
    counter_db(db, rows)
    out = run("counters", db)
    assert "== plain path: 1 dispatches" in out and "== batched path: 1 dispatches" in out
    line = [x for x in out.splitlines() if "k_select_sum" in x][0].split()
    assert line[3] == "50.0" and line[4] == "64" and line[5] == "0.100" and line[6] == "0.500"


def test_traffic_scaled_by_copy_calibration(tmp_path):
    neg = "void at::native::vectorized_elementwise_kernel<4, at::native::neg_kernel_cuda(x)>(int)"
    f = str(tmp_path / "f.db")
    w = str(tmp_path / "w.db")
    # the copy reads and writes 1 GiB; FETCH_SIZE counts half the bytes read, WRITE_SIZE all
    counter_db(f, [(1, neg, "FETCH_SIZE", 2.0 ** 30 / 2 / 1024, 1),
                   (2, "k_select_sum_planes_run(x)", "FETCH_SIZE", 2e9 / 1024, 1)])
    counter_db(w, [(1, neg, "WRITE_SIZE", 2.0 ** 30 / 1024, 1),
                   (2, "k_select_sum_planes_run(x)", "WRITE_SIZE", 3e9 / 1024, 1)])
    line = tmp_path / "bench.json"
    line.write_text("[bench] log line\n" + json.dumps({"copy_calibration_bytes": {"read": 2 ** 30, "written": 2 ** 30}}))
    out = run("traffic", f, w, str(line))
    assert "2.0000 bytes read per counted FETCH_SIZE byte, 1.0000 written" in out
    row = [x for x in out.splitlines() if x.strip().startswith("k_select_sum_planes_run")][0].split()
    assert row[2] == "4.000" and row[3] == "3.000"


def test_usage_without_arguments():
    r = subprocess.run([sys.executable, TOOL], capture_output=True, text=True)
    assert r.returncode == 2 and "profile_summary.py kernels" in r.stdout
