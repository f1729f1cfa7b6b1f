"""Host logic of the profile summaries the benchmark reads (no GPU): kernel
statistics of a trace, counter averages per dispatch, the traffic scaling by
the copy kernel of known size, and the per-entry tile and source-hash checks
of bench.py, on small synthetic rocprofv3-like databases."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2608_15249_amd import rocprof_summary as R  # noqa: E402

PUSH = "void apic::(anonymous namespace)::k_step_push<true, 2, 3, 1, false, false, true>(apic::Geo, ...)"
COUNT = "void apic::(anonymous namespace)::k_step_count<true, 2, 3, 1, false, false>(apic::Geo, ...)"
COPY = "void apic::(anonymous namespace)::k_copy_bytes(char const*, char*, long)"


def _trace_db(path):
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, start integer, end integer)")
    rows = []
    t = 0
    for i in range(6):                       # push durations 100..150 us, count 10 us
        rows.append((PUSH, t, t + 1000 * (100 + 10 * i)))
        t += 200000
        rows.append((COUNT, t, t + 10000))
        t += 20000
    con.executemany("insert into kernels values (?, ?, ?)", rows)
    con.commit()
    con.close()


def _pmc_db(path, counter, per_dispatch):
    """per_dispatch: [(kernel name, [values of the counter instances])]."""
    con = sqlite3.connect(path)
    con.execute("create table pmc_events (name text, dispatch_id integer, counter_name text, counter_value real)")
    rows = []
    for did, (name, vals) in enumerate(per_dispatch):
        for v in vals:
            rows.append((name, did, counter, v))
    con.executemany("insert into pmc_events values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()


def test_kernel_stats_and_names(tmp_path):
    db = str(tmp_path / "t.db")
    _trace_db(db)
    st = {n: (c, avg, tot, tail) for n, c, avg, tot, tail in R.kernel_stats(db, last=2)}
    push = "k_step_push<true, 2, 3, 1, false, false, true>"
    assert set(st) == {push, "k_step_count<true, 2, 3, 1, false, false>"}
    c, avg, tot, tail = st[push]
    assert c == 6 and avg == pytest.approx(125.0) and tot == pytest.approx(0.75) and tail == pytest.approx(145.0)
    # sorted by total time: the push first
    assert R.kernel_stats(db)[0][0] == push


def test_traffic_scaling_and_per_entry_tile(tmp_path, monkeypatch):
    copy = 1 << 20
    fdb, wdb = str(tmp_path / "f.db"), str(tmp_path / "w.db")
    # FETCH_SIZE reads half the copy's bytes (in KiB, split over two instances), WRITE_SIZE all of them
    _pmc_db(fdb, "FETCH_SIZE", [(COPY, [copy / 4096, copy / 4096]), (PUSH, [300.0, 100.0]), (PUSH, [250.0, 150.0]),
                                (COUNT, [10.0])])
    _pmc_db(wdb, "WRITE_SIZE", [(COPY, [copy / 1024]), (PUSH, [500.0]), (PUSH, [500.0]), (COUNT, [0.0])])
    out = str(tmp_path / "traffic.json")
    for tag, tile in (("mixed", "32x32"), ("fp64", "32x16")):
        subprocess.run([sys.executable, "-m", "paper_2608_15249_amd.rocprof_summary", "traffic", fdb, wdb,
                        "--kernel", "k_step", "--copy-bytes", str(copy), "--tag", tag, "--merge-into", out,
                        "--tile", tile, "--main", "k_step_push", "--cmd", "synthetic"],
                       cwd=ROOT, check=True, capture_output=True)
    d = json.load(open(out))
    assert d["kernel_src_sha"] == R.kernel_source_sha()
    e = d["mixed"]
    assert e["tile"] == [32, 32] and d["fp64"]["tile"] == [32, 16]
    assert e["detail"]["fetch_scale"] == pytest.approx(2.0) and e["detail"]["write_scale"] == pytest.approx(1.0)
    # push: 400 KiB fetched x 2 + 500 KiB written per dispatch
    assert e["hbm_bytes_per_launch"] == pytest.approx((400 * 2 + 500) * 1024.0)
    assert e["kernel"].startswith("k_step_push")
    # the benchmark takes an entry only at its own tile and source hash
    import bench
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    json.dump(d, open(tmp_path / "profiles" / "step_push_w_traffic.json", "w"))
    assert bench.load_traffic("mixed", "w", [32, 32]) == pytest.approx((400 * 2 + 500) * 1024.0)
    assert bench.load_traffic("mixed", "w", [32, 16]) is None
    assert bench.load_traffic("fp64", "w", [32, 16]) is not None
    d["kernel_src_sha"] = "0" * 16
    json.dump(d, open(tmp_path / "profiles" / "step_push_w_traffic.json", "w"))
    assert bench.load_traffic("mixed", "w", [32, 32]) is None


def test_counters_average_over_dispatches(tmp_path):
    a, b = str(tmp_path / "a.db"), str(tmp_path / "b.db")
    _pmc_db(a, "SQ_WAVES", [(PUSH, [2048.0, 2048.0]), (PUSH, [2048.0, 2048.0]), (COUNT, [7.0])])
    _pmc_db(b, "SQ_INSTS_VALU", [(PUSH, [10.0]), (PUSH, [30.0])])
    out = str(tmp_path / "c.json")
    subprocess.run([sys.executable, "-m", "paper_2608_15249_amd.rocprof_summary", "counters", a, b, "--kernel",
                    "k_step_push", "--tag", "mixed_sq", "--merge-into", out, "--tile", "16x8x8"],
                   cwd=ROOT, check=True, capture_output=True)
    d = json.load(open(out))
    e = d["mixed_sq"]
    assert e["tile"] == [16, 8, 8]
    assert e["per_launch"] == {"SQ_WAVES": 4096.0, "SQ_INSTS_VALU": 20.0}
