"""profsum --bench: the text tables of bench.py's JSON lines (benchmark,
--sweep and --batched forms) carry the figures of the line they format."""

import json
import os
import subprocess
import sys

from paper_1104_0737_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _op(ms):
    return {"ms": ms, "algo_GBps": 2000.0 + ms, "frac_hbm_peak": 0.25}


BENCH = {"metric": "m", "value": 6.5e9, "unit": "site·RHS/s", "steps": 3, "ms_per_step": 917.6, "iterations": 6,
         "max_true_res": 1.9e-11, "config": {"workload": "32x32x32x64 test"},
         "tts_per_rhs_s": {"mixed": 0.0765, "fp64": 0.1626, "fp64_over_mixed": 2.125},
         "other_sap_prec_solve": {"sap_prec": "fp16s", "seconds": 0.778, "iterations": 6, "max_true_res": 2.8e-11},
         "ssor_domain_solve": {"seconds": 0.545, "iterations": 4, "max_true_res": 4.4e-13},
         "dslash": {"fp64": _op(3.935), "fp32": _op(1.904), "fp16s": _op(1.447)},
         "roofline": {"kernel": "mr_dslash", "launches": 384, "avg_launch_ms": 0.792, "bytes_per_launch": 2.416e9,
                      "achieved": 3050.6, "unit": "GB/s", "frac": 0.3813, "peak": 8000.0, "traffic": 3.47e9,
                      "traffic_over_algorithmic": 1.437},
         "cpu_baseline": {"kind": "oracle", "cores": 1, "value": 1.33e6, "unit": "site·RHS/s", "sample": "slab"}}

SWEEP = {"workload": "sweep test", "sweep": [
    {"L": L, "blocks": 12 // L, "dslash": {"fp64": _op(0.5 * L), "fp32": _op(0.3 * L), "fp16s": _op(0.2 * L)},
     "mixed_mr": {"seconds": 2.0 / L, "iterations": [5, 6]}, "fp64_mr": {"seconds": 3.0 / L, "iterations": [6]},
     "mixed_ssor": {"seconds": 1.0 / L, "iterations": [3, 4]},
     "gain_vs_L1": {"mixed_mr": float(L), "fp64_mr": float(L), "mixed_ssor": float(L)}} for L in (1, 12)]}

BATCHED = {"metric": "batched", "config": {"workload": "48 systems"}, "ms_per_step": 738.7, "steps": 3,
           "value": 476.5, "unit": "RHS/s", "converged": True, "max_true_res": 9.98e-11, "separate_handles_s": 0.752,
           "sequential_s": 0.859, "fused_over_sequential": 1.163, "iterations": {"8x8x8x8": [3, 5]}}


def test_benchmark_line():
    t = profsum.bench_table(BENCH)
    for s in ("0.918 s", "6 iterations", "(2.12x)", "(fp16s) 0.778 s", "0.545 s", "3.935 ms", "1.447 ms",
              "384 launches of 0.792 ms", "0.381 of 8000", "3.470 GB (1.44x)", "1.330e+06"):
        assert s in t, s
    nt = dict(BENCH, roofline=dict(BENCH["roofline"], traffic=None))
    assert "counter traffic null" in profsum.bench_table(nt)


def test_sweep_and_batched_lines():
    t = profsum.bench_table(SWEEP).splitlines()
    assert len(t) == 4 and t[2].split()[:2] == ["1", "12"] and t[3].split()[:2] == ["12", "1"]
    assert "5-6" in t[2] and "12.00" in t[3]
    b = profsum.bench_table(BATCHED)
    for s in ("0.739 s per step", "476.5 RHS/s", "0.752 s", "0.859 s", "1.163x", "8x8x8x8: 3-5"):
        assert s in b, s


def test_cli(tmp_path):
    f = tmp_path / "b.json"
    f.write_text("[log line]\n" + json.dumps(BATCHED) + "\n")
    r = subprocess.run([sys.executable, "-m", "paper_1104_0737_amd.profsum", "--bench", str(f)], cwd=ROOT,
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and "1.163x" in r.stdout
