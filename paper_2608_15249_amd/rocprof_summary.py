"""Summaries of rocprofv3 result databases (kernel trace and PMC counters).

Usage:
  python -m paper_2608_15249_amd.rocprof_summary trace <results.db> [--cmd "..."] [--last N]
  python -m paper_2608_15249_amd.rocprof_summary counters <pass1.db> [<pass2.db> ...] --kernel k_step_push \
        --tag mixed --merge-into profiles/step_push_<workload>_counters.json --tile 32x32 [--cmd "..."]
  python -m paper_2608_15249_amd.rocprof_summary traffic <fetch.db> <write.db> \
        --kernel k_step --copy-bytes N [--cmd "..."] [--tag mixed] \
        [--merge-into profiles/step_push_<workload>_traffic.json --tile 8x8 --main k_step_push]

`trace` prints per-kernel call counts and average/total durations.
`counters` averages every counter of one or more PMC passes per dispatch of
the named kernel (the timed launches of the run) and stores them, with the
bucket tile of the run, under the tag in a file keyed by the source hash
(the benchmark reads the atomic counts from there). `traffic` turns FETCH_SIZE / WRITE_SIZE (KiB per dispatch, summed over the counter
instances of a dispatch) into HBM bytes per dispatch of the named kernel,
each scaled by the factor that makes the same counter read the known byte
count of the plain copy kernel (k_copy_bytes) of the same run. With
--merge-into the result is stored under its tag, with the bucket tile of the
run, in a JSON file keyed by the hash of the step kernels' sources: what the
benchmark checks before it reports the counted traffic.
"""
from __future__ import annotations

import argparse
import collections
import hashlib
import json
import os
import re
import sqlite3

_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
KERNEL_SOURCES = ("apic_kernels.hip", "apic_device.h", "apic_internal.h", "apic_em.h")


def _code_only(text: str) -> str:
    """C++ source without its comments, trailing blanks and empty lines
    (string and character literals kept as written)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    lines = (ln.rstrip() for ln in "".join(out).split("\n"))
    return "\n".join(ln for ln in lines if ln)


def kernel_source_sha() -> str:
    """Hash of the step kernels' code (a counter run is valid for this code
    only; comments and blank space do not enter it)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(_CSRC, f), encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def _short(name: str) -> str:
    n = name.replace("void ", "").replace("apic::(anonymous namespace)::", "")
    m = re.match(r"([A-Za-z_0-9]+)(<[^>]*>)?", n)
    return (m.group(1) + (m.group(2) or "")) if m else n[:60]


def kernel_stats(db: str, last: int = 0):
    """(kernel, calls, avg_us, total_ms, avg_us of the last `last` dispatches
    by start time or None), sorted by total time."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end from kernels order by start").fetchall()
    per = collections.defaultdict(list)
    for n, st, en in rows:
        per[_short(n)].append((en - st) / 1e3)
    out = []
    for n, d in per.items():
        tail = d[-last:] if last and len(d) >= last else None
        out.append((n, len(d), sum(d) / len(d), sum(d) / 1e3, None if tail is None else sum(tail) / len(tail)))
    out.sort(key=lambda r: -r[3])
    return out


def pmc_per_dispatch(db: str, counter: str):
    """{kernel short name: [value per dispatch]} summed over counter instances."""
    con = sqlite3.connect(db)
    per = collections.defaultdict(float)
    names = {}
    for name, did, cn, cv in con.execute("select name, dispatch_id, counter_name, counter_value from pmc_events"):
        if cn != counter:
            continue
        per[did] += cv
        names[did] = _short(name)
    out = collections.defaultdict(list)
    for did, v in per.items():
        out[names[did]].append(v)
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--cmd", default="")
    t.add_argument("--last", type=int, default=0,
                   help="also average the last N dispatches of each kernel (the timed steps of a run)")
    q = sub.add_parser("counters")
    q.add_argument("dbs", nargs="+")
    q.add_argument("--kernel", required=True)
    q.add_argument("--tag", required=True)
    q.add_argument("--merge-into", required=True)
    q.add_argument("--tile", default="")
    q.add_argument("--cmd", default="")
    f = sub.add_parser("traffic")
    f.add_argument("fetch_db")
    f.add_argument("write_db")
    f.add_argument("--kernel", required=True)
    f.add_argument("--copy-bytes", type=float, required=True)
    f.add_argument("--cmd", default="")
    f.add_argument("--tag", default="")
    f.add_argument("--merge-into", default="")
    f.add_argument("--tile", default="")
    f.add_argument("--main", default="", help="kernel (name prefix) whose bytes are the headline")
    a = ap.parse_args()
    if a.cmd_name == "counters":
        per = {}
        name = None
        for db in a.dbs:
            con = sqlite3.connect(db)
            cn_names = sorted({r[0] for r in con.execute("select distinct counter_name from pmc_events")})
            for cn in cn_names:
                vals = pmc_per_dispatch(db, cn)
                ks = [k for k in vals if k.startswith(a.kernel)]
                if not ks:
                    continue
                name = ks[0]
                v = vals[ks[0]]
                per[cn] = sum(v) / len(v)
        sha = kernel_source_sha()
        tile = [int(v) for v in a.tile.lower().split("x")] if a.tile else []
        d = {}
        if os.path.exists(a.merge_into):
            with open(a.merge_into) as fh:
                d = json.load(fh)
            if d.get("kernel_src_sha") != sha:
                d = {}
        d["kernel_src_sha"] = sha
        d["note"] = ("counter values per dispatch of the kernel, averaged over its dispatches in the profiled run; "
                     "each entry with the bucket tile of its run")
        d[a.tag] = {"kernel": name, "tile": tile, "per_launch": per, "command": a.cmd}
        with open(a.merge_into, "w") as fh:
            json.dump(d, fh, indent=1)
        print(json.dumps(d[a.tag], indent=1))
        return
    if a.cmd_name == "trace":
        if a.cmd:
            print("command: %s" % a.cmd)
        head = "%-46s %7s %12s %12s" % ("kernel", "calls", "avg_us", "total_ms")
        if a.last:
            head += " %14s" % ("avg_last%d_us" % a.last)
        print(head)
        for n, c, avg, tot, tail in kernel_stats(a.db, a.last):
            line = "%-46s %7d %12.2f %12.3f" % (n[:46], c, avg, tot)
            if a.last:
                line += " %14s" % ("" if tail is None else "%.2f" % tail)
            print(line)
        return
    fe = pmc_per_dispatch(a.fetch_db, "FETCH_SIZE")
    wr = pmc_per_dispatch(a.write_db, "WRITE_SIZE")
    cf = [v for k, v in fe.items() if k.startswith("k_copy_bytes")]
    cw = [v for k, v in wr.items() if k.startswith("k_copy_bytes")]
    copy_f = max(x for vals in cf for x in vals) * 1024.0
    copy_w = max(x for vals in cw for x in vals) * 1024.0
    ff = a.copy_bytes / copy_f
    fw = a.copy_bytes / copy_w
    res = {"command": a.cmd, "tag": a.tag, "fetch_scale": ff, "write_scale": fw, "copy_bytes": a.copy_bytes,
           "kernels": {}}
    for k in sorted(set(fe) | set(wr)):
        if not k.startswith(a.kernel):
            continue
        fk = sum(fe[k]) / len(fe[k]) * 1024.0 * ff
        wk = sum(wr[k]) / len(wr[k]) * 1024.0 * fw
        res["kernels"][k] = {"fetch_bytes": fk, "write_bytes": wk, "hbm_bytes_per_launch": fk + wk,
                             "dispatches": len(fe[k])}
    print(json.dumps(res, indent=1))
    if a.merge_into:
        sha = kernel_source_sha()
        tile = [int(v) for v in a.tile.lower().split("x")] if a.tile else []
        d = {}
        if os.path.exists(a.merge_into):
            with open(a.merge_into) as fh:
                d = json.load(fh)
            if d.get("kernel_src_sha") != sha:
                d = {}
        d["kernel_src_sha"] = sha
        d["note"] = ("HBM bytes per launch of the step kernels; FETCH_SIZE and WRITE_SIZE (KiB per dispatch, "
                     "summed over counter instances) scaled so that the plain copy kernel k_copy_bytes of the "
                     "same run reads/writes its known size; each entry with the bucket tile of its run")
        main_k = [k for k in res["kernels"] if k.startswith(a.main or a.kernel)]
        d[a.tag] = {"kernel": main_k[0] if main_k else None, "tile": tile,
                    "hbm_bytes_per_launch": res["kernels"][main_k[0]]["hbm_bytes_per_launch"] if main_k else None,
                    "detail": res}
        with open(a.merge_into, "w") as fh:
            json.dump(d, fh, indent=1)


if __name__ == "__main__":
    main()
