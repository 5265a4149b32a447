"""Summarise rocprofv3 SQLite output (kernel trace and PMC counters) as text.

usage: python -m paper_1104_0737_amd.profsum DB [DB ...] [--match SUBSTR]
Kernel-trace databases print calls and average/total duration per kernel;
counter databases print the average counter value per dispatch per kernel.
"""

from __future__ import annotations

import argparse
import re
import sqlite3
from collections import defaultdict


def short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    name = re.sub(r"\(.*$", "", name)
    name = name.replace("mbbs::", "").replace("void ", "")
    return name if len(name) < 90 else name[:87] + "..."


def kernel_stats(db):
    c = sqlite3.connect(db)
    rows = c.execute("select name, total_calls, total_duration, average from top_kernels").fetchall()
    # top_kernels reports durations in microseconds
    return [(short(n), k, tot / 1e3, avg) for n, k, tot, avg in rows]


def counters(db):
    c = sqlite3.connect(db)
    acc = defaultdict(list)
    for name, cname, val in c.execute("select kernel_name, counter_name, value from counters_collection"):
        acc[(short(name), cname)].append(val)
    return [(k[0], k[1], len(v), sum(v) / len(v)) for k, v in acc.items()]


def traffic(fetch_db, write_db, cfetch_db, cwrite_db, classes, copy_bytes=4 << 30):
    """HBM bytes per launch of the named kernels from a FETCH_SIZE and a
    WRITE_SIZE run (KiB per dispatch), each scaled by what the same counter
    reads for a plain device copy of `copy_bytes` bytes.  classes maps a
    kernel class to its kernel name, or to several names joined by '+' (the
    class's figure is then the mean over all their dispatches).  Returns a
    JSON-ready dict that also records the hash of the sources the counters
    were taken with."""
    from .build import source_hash

    def avg(db, cname, kname):
        vals = [(n, v) for k, c, n, v in counters(db) if c == cname and k == kname]
        return vals[0] if vals else (0, None)
    copy = "__amd_rocclr_copyBuffer"
    rs = copy_bytes / 1024 / avg(cfetch_db, "FETCH_SIZE", copy)[1]
    ws = copy_bytes / 1024 / avg(cwrite_db, "WRITE_SIZE", copy)[1]
    out = {"source_hash": source_hash(), "read_scale": rs, "write_scale": ws, "classes": {}}
    for cls, knames in classes.items():
        parts, nf, nw, fs, wsum = [], 0, 0, 0.0, 0.0
        for kname in knames.split("+"):
            (n1, f), (n2, w) = avg(fetch_db, "FETCH_SIZE", kname), avg(write_db, "WRITE_SIZE", kname)
            if f is None or w is None:
                parts = None
                break
            parts.append({"kernel": kname, "dispatches": n1, "fetch_kib": f, "write_kib": w})
            nf, nw, fs, wsum = nf + n1, nw + n2, fs + n1 * f, wsum + n2 * w
        if not parts:
            continue
        f, w = fs / nf, wsum / nw
        out["classes"][cls] = {"kernel": knames, "fetch_kib": f, "write_kib": w,
                               "bytes": f * 1024 * rs + w * 1024 * ws}
        if len(parts) > 1:
            out["classes"][cls]["parts"] = parts
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db", nargs="*")
    ap.add_argument("--match", default="")
    ap.add_argument("--traffic", nargs=4, metavar=("FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB"),
                    help="print per-launch HBM traffic of --kernel CLASS=NAME pairs as JSON")
    ap.add_argument("--kernel", action="append", default=[])
    a = ap.parse_args()
    if a.traffic:
        import json
        classes = dict(kv.split("=", 1) for kv in a.kernel)
        print(json.dumps(traffic(*a.traffic, classes), indent=1))
        return
    for db in a.db:
        c = sqlite3.connect(db)
        has_pmc = c.execute("select count(*) from counters_collection").fetchone()[0] > 0
        print(f"# {db}")
        if has_pmc:
            print(f"{'kernel':90s} {'counter':12s} {'n':>4s} {'avg/dispatch':>16s}")
            for k, cn, n, v in counters(db):
                if a.match in k:
                    print(f"{k:90s} {cn:12s} {n:4d} {v:16.1f}")
        else:
            print(f"{'kernel':90s} {'calls':>6s} {'total ms':>10s} {'avg us':>10s}")
            for k, n, tot, avg in kernel_stats(db):
                if a.match in k:
                    print(f"{k:90s} {n:6d} {tot:10.3f} {avg:10.1f}")


if __name__ == "__main__":
    main()
