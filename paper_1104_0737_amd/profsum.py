"""Summarise rocprofv3 SQLite output (kernel trace and PMC counters) as text.

usage: python -m paper_1104_0737_amd.profsum DB [DB ...] [--match SUBSTR]
       python -m paper_1104_0737_amd.profsum --bench JSON   (a bench.py line: benchmark, --sweep or --batched)
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


def bench_table(line: dict) -> str:
    """Text table of a bench.py --sweep line (per L: operator times and solve
    times), of a --batched line (fused, separate-handle and sequential times,
    iterations per lattice) or of a benchmark line (solves and operators)."""
    out = []
    if "sweep" in line:
        out.append(f"# {line['workload']}")
        out.append(f"{'L':>3s} {'blocks':>6s} {'op FP64 ms':>10s} {'FP64 GB/s':>9s} {'op FP32 ms':>10s} "
                   f"{'op FP16S ms':>11s} {'mixed MR s':>10s} {'FP64 MR s':>9s} {'mixed SSOR s':>12s} "
                   f"{'it MR':>6s} {'it SSOR':>7s} {'gain MR / FP64 / SSOR vs L=1':>28s}")
        for r in line["sweep"]:
            d, g = r["dslash"], r["gain_vs_L1"]
            it = lambda k: f"{min(r[k]['iterations'])}-{max(r[k]['iterations'])}"
            out.append(f"{r['L']:3d} {r['blocks']:6d} {d['fp64']['ms']:10.3f} {d['fp64']['algo_GBps']:9.0f} "
                       f"{d['fp32']['ms']:10.3f} {d['fp16s']['ms']:11.3f} {r['mixed_mr']['seconds']:10.3f} "
                       f"{r['fp64_mr']['seconds']:9.3f} {r['mixed_ssor']['seconds']:12.3f} {it('mixed_mr'):>6s} "
                       f"{it('mixed_ssor'):>7s} {g['mixed_mr']:10.2f} {g['fp64_mr']:6.2f} {g['mixed_ssor']:6.2f}")
    elif "dslash" in line:
        out.append(f"# {line['config']['workload']}")
        out.append(f"mixed solve           {line['ms_per_step'] / 1e3:.3f} s per step ({line['steps']} steps), "
                   f"{line['iterations']} iterations, max true residual {line['max_true_res']:.2e}; "
                   f"{line['value']:.3e} {line['unit']}")
        t = line.get("tts_per_rhs_s") or {}
        if "fp64" in t:
            out.append(f"per RHS               mixed {t['mixed']:.4f} s, all-FP64 {t['fp64']:.4f} s "
                       f"({t['fp64_over_mixed']:.2f}x)")
        for key, name in (("other_sap_prec_solve", "other SAP storage"), ("ssor_domain_solve", "SSOR domains")):
            o = line.get(key)
            if o:
                tag = f" ({o['sap_prec']})" if "sap_prec" in o else ""
                out.append(f"{name + tag:21s} {o['seconds']:.3f} s, {o['iterations']} iterations, "
                           f"max true residual {o['max_true_res']:.2e}")
        for prec, d in line["dslash"].items():
            out.append(f"operator {prec:12s} {d['ms']:.3f} ms, {d['algo_GBps']:.0f} GB/s algorithmic "
                       f"({100 * d['frac_hbm_peak']:.0f} % of HBM peak)")
        r = line.get("roofline")
        if r:
            tr = (f", counter traffic {r['traffic'] / 1e9:.3f} GB ({r['traffic_over_algorithmic']:.2f}x)"
                  if r.get("traffic") else ", counter traffic null")
            out.append(f"roofline {r['kernel']}: {r['launches']} launches of {r['avg_launch_ms']:.3f} ms, "
                       f"{r['bytes_per_launch'] / 1e9:.3f} GB algorithmic each, {r['achieved']:.0f} {r['unit']} "
                       f"= {r['frac']:.3f} of {r['peak']:.0f}{tr}")
        c = line.get("cpu_baseline")
        if c:
            out.append(f"cpu baseline ({c['kind']}, {c['cores']} core): {c['value']:.3e} {c['unit']}; {c['sample']}")
    else:
        out.append(f"# {line['metric']}: {line['config']['workload']}")
        out.append(f"fused batched solve   {line['ms_per_step'] / 1e3:.3f} s per step ({line['steps']} steps), "
                   f"{line['value']:.1f} {line['unit']}, all converged: {line['converged']}, "
                   f"max true residual {line['max_true_res']:.2e}")
        out.append(f"separate handles      {line['separate_handles_s']:.3f} s (one batched call)")
        out.append(f"one system at a time  {line['sequential_s']:.3f} s")
        out.append(f"fused / sequential    {line['fused_over_sequential']:.3f}x")
        for k, v in line["iterations"].items():
            out.append(f"iterations {k}: {v[0]}-{v[1]}")
    return "\n".join(out)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("db", nargs="*")
    ap.add_argument("--match", default="")
    ap.add_argument("--traffic", nargs=4, metavar=("FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB"),
                    help="print per-launch HBM traffic of --kernel CLASS=NAME pairs as JSON")
    ap.add_argument("--kernel", action="append", default=[])
    ap.add_argument("--bench", default=None, help="print a table of a bench.py JSON line (benchmark, --sweep or --batched)")
    a = ap.parse_args()
    if a.bench:
        import json
        with open(a.bench) as f:
            print(bench_table(json.loads(f.read().strip().splitlines()[-1])))
        return
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
