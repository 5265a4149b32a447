"""Benchmark: SAP-preconditioned modified block BiCGSTAB on a 32^3 x 64 lattice.

One step is one mixed-precision solve (outer recurrences, Gram products,
Cholesky QR, L x L solves and true residual in FP64; SAP with its MR domain
solves in FP32) of D X = B for L = 12 point sources (all spin-colour
components at one seeded site), tolerance 1e-10 on every column, with the
inputs resident in HBM when the timed region starts.  Synthetic random SU(3)
links (eps = 0.2, kappa = 0.1240) stand in for the paper's gauge
configurations.  Reported beside it: the operator's stand-alone rate in FP64,
FP32 and FP16 storage, the all-FP64 solve's time per right-hand side, the
dominant kernel's roofline (event-timed inside the timed solves), and the CPU
oracle's operator rate on a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Dslash site·RHS/s (HBM GB/s) + time-to-solution/RHS, mixed vs FP64 @1e-10"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--L", type=int, default=12)
    ap.add_argument("--dims", type=str, default="32,32,32,64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-solve", action="store_true")
    ap.add_argument("--dslash-reps", type=int, default=20)
    ap.add_argument("--only-dslash", action="store_true", help="stand-alone operator timing only")
    ap.add_argument("--skip-dslash", action="store_true", help="no stand-alone operator timing")
    ap.add_argument("--no-tune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--profile", type=int, default=1, help="event-time kernel classes in the timed solves")
    ap.add_argument("--sap-prec", choices=("fp32", "fp16s"), default="fp32",
                    help="storage precision of the SAP preconditioner in the mixed solve")
    ap.add_argument("--apply-tuning", default=None,
                    help="apply the launch settings of an earlier run's JSON line instead of tuning")
    ap.add_argument("--csw", type=float, default=0.0,
                    help="clover coefficient: O(a)-improved operator with Jacobi preconditioning (0: Wilson)")
    ap.add_argument("--domain-solver", choices=("mr", "ssor"), default="mr",
                    help="SAP domain solver: nmr MR steps, or SSOR (N_SSOR, omega) as in the paper")
    ap.add_argument("--nssor", type=int, default=1)
    ap.add_argument("--ssor-omega", type=float, default=1.26)
    ap.add_argument("--sweep", action="store_true",
                    help="L sweep over 1,2,3,4,6,12 (12 point sources in 12/L blocks), operator and solves")
    ap.add_argument("--batched", action="store_true",
                    help="48 independent systems of uneven size solved together (batched form)")
    ap.add_argument("--graph-iters", type=int, default=4)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a device-to-device copy of 4 GiB (HBM counter calibration)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(cls, L, dims, block, ncy, nmr, sap_prec="fp32", nssor=1, clover=False, once=False,
                      tiled=False):
    """Compulsory HBM bytes of one launch of a kernel class, averaged over the
    launches of one SAP application where they differ.  SAP storage: FP32
    8-byte complex and 72-byte link, or FP16 storage 4-byte complex plus one
    4-byte scale per site and column and 36-byte link; psi is FP32; the outer
    operator is FP64 (16-byte complex, 144-byte link).

    dslash64   whole lattice: read X, write Y, 4 links per site.
    mr_dslash  one colour (V/2 sites): read r, write w, 4 links per site.
    mr_update  one colour: read r and psi, write psi; while r is still
               needed also read w and write r; the first step of the first
               cycle assigns psi (no psi read).
    With psi formed once per domain solve (once=True) sap_resid has no pass
    on the first colour of the first cycle, and the MR steps only
    carry the residual: mr_update is then nmr - 1 residual steps (read r and
    w, write the next r) and one psi pass (read r_0 and the first nmr - 1 A r,
    read psi except in the first cycle, write psi); the last MR step of the
    tiled stencil (tiled=True) stores no A r, since only its omega is used.
    sap_resid  one colour: read eta, write r; except on the first half-sweep
               also read psi on the colour and on the other colour's sites
               that touch it (a fraction f of them), and 4 links per site.
    ssor       one colour, all sweeps, SAP residual included: N_SSOR = 1 moves
               10 storage fields (eta->a, a->b, a,b->r,a, a->b), psi (the
               residual's stencil as in sap_resid, then read + write, assign
               in the first cycle), 4 links per site and sweep plus the
               residual's; N_SSOR = 0 moves 4 (eta->a, a->b), 2 sweeps.
    With the clover term every stencil pass also reads the packed site
    inverse (72 reals per site: FP64 576 bytes, FP32 288 bytes).
    """
    V = int(np.prod(dims))
    Vh = V // 2
    sp = 12 * L * 8 if sap_prec == "fp32" else 12 * L * 4 + 4 * L   # storage spinor row block
    ps = 12 * L * 8                                                  # psi (FP32)
    lk = 72 if sap_prec == "fp32" else 36
    cl = 288 if clover else 0
    if cls == "dslash64":
        return V * ((48 * L + 72) * 8 + (576 if clover else 0))
    if cls == "mr_dslash":
        if once and tiled:
            return Vh * (sp + 4 * lk + cl) + Vh * sp * (nmr - 1) / nmr
        return Vh * (2 * sp + 4 * lk + cl)
    if cls == "mr_update" and once:
        tot = 0
        for cy in range(ncy):
            tot += (nmr - 1) * 3 * sp + nmr * sp + (ps if cy == 0 else 2 * ps)
        return Vh * tot / (ncy * nmr)
    if cls == "mr_update":
        tot = 0
        for cy in range(ncy):
            for it in range(nmr):
                b = sp + ps + (0 if (cy == 0 and it == 0) else ps) + (2 * sp if it + 1 < nmr else 0)
                tot += 2 * Vh * b      # both colours
        return tot / (2 * ncy * nmr)
    if cls == "sap_resid":
        inner = int(np.prod([b - 2 for b in block]))
        f = 1 - inner / int(np.prod(block))  # sites of a domain that touch another domain
        # with psi formed once, the first colour of the first cycle has no
        # residual pass (its domain solves read eta)
        tot = (1 if once else 2) * (2 * Vh * sp)         # first cycle, colour 0 and 1: eta, r
        tot += Vh * (f * ps + 4 * lk)                    # first cycle, colour 1: psi of colour 0
        tot += 2 * (ncy - 1) * Vh * (2 * sp + (1 + f) * ps + 4 * lk)
        tot += (2 * ncy - 1) * Vh * cl                   # every half-sweep but the first
        return tot / (2 * ncy - (1 if once else 0))
    if cls == "ssor":
        # the SAP residual is formed inside the first sweep
        inner = int(np.prod([b - 2 for b in block]))
        f = 1 - inner / int(np.prod(block))
        fields, sweeps = (10, 4) if nssor == 1 else (4, 2)
        tot = 0
        for cy in range(ncy):
            for col in range(2):
                mode = 2 if cy > 0 else col
                resid = 0 if mode == 0 else (f * ps if mode == 1 else (1 + f) * ps) + 4 * lk + cl
                upd = ps if cy == 0 else 2 * ps
                tot += Vh * (fields * sp + resid + upd + sweeps * (4 * lk + cl))
        return tot / (2 * ncy)
    return None


def measured_traffic(cls, dims, L, sap_prec, clover=False):
    """HBM bytes per launch of a kernel class from the committed counter
    summary (FETCH_SIZE / WRITE_SIZE, copy-calibrated) for this workload; None
    if there is none or the library's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_32x32x32x64_L12.json")
    if (tuple(dims) != (32, 32, 32, 64) or L != 12 or sap_prec != "fp32" or clover
            or not os.path.exists(path)):
        return None
    from paper_1104_0737_amd.build import source_hash
    with open(path) as f:
        t = json.load(f)
    if t.get("source_hash") != source_hash() or cls not in t["classes"]:
        return None
    return t["classes"][cls]["bytes"]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "sharding one system over several GPUs (by whole SAP domains) is designed but not built.", flush=True)
        sys.exit(1)
    import torch
    from paper_1104_0737_amd import binding as B
    from paper_1104_0737_amd import configs, model

    if args.copy_calibration:
        # a plain copy of known size: 4 GiB read, 4 GiB written per launch
        a = torch.empty(1 << 29, dtype=torch.float64, device="cuda:0").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8}), flush=True)
        return

    if args.batched:
        return batched_main(args)
    if args.sweep:
        return sweep_main(args)

    dims = tuple(int(x) for x in args.dims.split(","))
    cfg = configs.c4(L=args.L)
    cfg.dims = dims
    V = int(np.prod(dims))
    L = args.L
    N = 12 * V
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)

    log(f"generating links for {dims}")
    t0 = time.time()
    U = cfg.gauge()
    log(f"links ready in {time.time() - t0:.1f}s")
    Ud = torch.from_numpy(U).to(dev)
    lat = B.mbbs_lattice_create(dims, cfg.block, Ud, cfg.kappa, cfg.phases, stream=stream)
    if args.csw:
        B.mbbs_lattice_set_clover(lat, args.csw, stream=stream)
        log(f"clover term set, c_sw = {args.csw}")
    del Ud

    # ------------------------------------------------------------ operator alone
    def time_dslash(prec):
        gen = torch.Generator(device=dev)
        gen.manual_seed(7)
        X = torch.randn((N, L), dtype=torch.complex128, device=dev, generator=gen)
        if prec == B.FP64:
            Xr, Yr, Xs, Ys = X, torch.empty_like(X), None, None
        else:
            dt = torch.float32 if prec == B.FP32 else torch.float16
            Xr = torch.empty((N, L, 2), dtype=dt, device=dev)
            Yr = torch.empty_like(Xr)
            Xs = torch.empty((V, L), dtype=torch.float32, device=dev) if prec == B.FP16S else None
            Ys = torch.empty_like(Xs) if Xs is not None else None
            B.mbbs_convert_to(prec, V, L, X, Xr, Xs, stream=stream)
        for _ in range(3):
            B.mbbs_apply_dirac_raw(lat, L, prec, Xr, Xs, Yr, Ys, stream=stream)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        for _ in range(args.dslash_reps):
            B.mbbs_apply_dirac_raw(lat, L, prec, Xr, Xs, Yr, Ys, stream=stream)
        ev1.record(stream)
        ev1.synchronize()
        ms = ev0.elapsed_time(ev1) / args.dslash_reps
        name = {B.FP64: "fp64", B.FP32: "fp32", B.FP16S: "fp16s"}[prec]
        by = model.dslash_bytes_per_site(L, name, bool(args.csw)) * V
        fl = model.dslash_flops_per_site(L) * V
        del X, Xr, Yr, Xs, Ys
        torch.cuda.empty_cache()
        return {"ms": ms, "site_rhs_per_s": V * L / (ms * 1e-3), "algo_GBps": by / (ms * 1e-3) / 1e9,
                "frac_hbm_peak": by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "TFLOPs": fl / (ms * 1e-3) / 1e12,
                "bytes_per_launch": by}

    # ------------------------------------------------------------ launch tuning
    tuning = {}
    dslash = {}
    if args.apply_tuning:
        # settings chosen by an earlier run (its JSON line), applied without
        # timing candidates: profiler runs then see only the kernels that run
        from paper_1104_0737_amd import autotune
        with open(args.apply_tuning) as f:
            prev = json.loads(f.read().strip().splitlines()[-1])["tuning"]
        for prec, name in ((B.FP64, "fp64"), (B.FP32, "fp32"), (B.FP16S, "fp16s")):
            t = prev[name]
            op = (t["group_cols"], t["block_threads"], t["split"], t["hop_pair"], t["nt_store"], t.get("chunk", 0),
                  t.get("tile", 0), 0, t.get("tile_cols", 0))
            autotune.apply(lat, prec, op)
            if not args.skip_dslash:
                dslash[name] = time_dslash(prec)
                dslash[name]["setting"] = list(op)
                log(f"  operator {name}: {dslash[name]['ms']:.3f} ms")
            if "sap" in t:
                autotune.apply(lat, prec, tuple(t["sap"]["setting"]))   # may set columns per thread
            tuning[name] = t
        log(f"applied tuning from {args.apply_tuning}")
    elif not args.no_tune:
        from paper_1104_0737_amd import autotune
        for prec, name in ((B.FP64, "fp64"), (B.FP32, "fp32"), (B.FP16S, "fp16s")):
            best, times = autotune.tune_operator(lat, V, L, prec, stream=stream)
            tuning[name] = {"group_cols": best[0], "block_threads": best[1], "split": best[2],
                            "hop_pair": best[3], "nt_store": best[4], "chunk": best[5] if len(best) > 5 else 0,
                            "tile": best[6] if len(best) > 6 else 0,
                            "tile_cols": best[8] if len(best) > 8 else 0,
                            "ms": round(times[best], 4), "worst_ms": round(max(times.values()), 4),
                            "classic_best_ms": round(min(v for k, v in times.items()
                                                         if k[2] == 0 and not (len(k) > 6 and k[6])), 4)}
            tiled_ms = [v for k, v in times.items() if len(k) > 6 and k[6]]
            if tiled_ms:
                tuning[name]["tiled_best_ms"] = round(min(tiled_ms), 4)
            log(f"tuned {name}: {best} ({times[best]:.3f} ms; "
                f"best classic {tuning[name]['classic_best_ms']:.3f} ms; worst {max(times.values()):.3f} ms)")
            if not args.skip_dslash:
                # the operator alone, in its fastest setting
                dslash[name] = time_dslash(prec)
                dslash[name]["setting"] = list(best)
                log(f"  operator {name}: {dslash[name]['ms']:.3f} ms, {dslash[name]['algo_GBps']:.0f} GB/s algorithmic")
            if prec != B.FP64:
                # the SAP kernels of this precision: split or one thread per site
                sbest, stimes = autotune.tune_sap(lat, V, L, prec, times, stream=stream)
                tuning[name]["sap"] = {"setting": list(sbest), "ms": {str(k): round(v, 3) for k, v in stimes.items()}}
                log(f"  SAP shape {sbest}: " + ", ".join(f"{k}: {v:.2f} ms" for k, v in stimes.items()))
        torch.cuda.empty_cache()

    for prec, name in () if args.skip_dslash or not args.no_tune or args.apply_tuning else ((B.FP64, "fp64"), (B.FP32, "fp32"),
                                                                        (B.FP16S, "fp16s")):
        log(f"operator {name}")
        dslash[name] = time_dslash(prec)
        log(f"  {dslash[name]['ms']:.3f} ms, {dslash[name]['algo_GBps']:.0f} GB/s algorithmic")
    if args.only_dslash:
        print(json.dumps({"dslash": dslash, "tuning": tuning}), flush=True)
        B.mbbs_lattice_destroy(lat)
        return

    # ------------------------------------------------------------ solves
    site = cfg.src_site()
    Bd = torch.zeros((N, L), dtype=torch.complex128, device=dev)
    for j in range(L):
        Bd[12 * site + cfg.comp0 + j, j] = 1.0
    Xd = torch.empty_like(Bd)

    sap_prec = {"fp32": B.FP32, "fp16s": B.FP16S}[args.sap_prec]

    def run_solve(sap_prec, profile):
        p = B.mbbs_solve_params_default(tol=cfg.tol, sap_prec=sap_prec, ncy=cfg.ncy, nmr=cfg.nmr,
                                        profile=profile, graph_iters=1,
                                        domain_solver=1 if args.domain_solver == "ssor" else 0,
                                        nssor=args.nssor, ssor_omega=args.ssor_omega)
        ws = torch.empty(B.mbbs_solve_workspace_size(lat, L, p), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        t = time.perf_counter()
        info = B.mbbs_solve(lat, L, Bd, Xd, p, ws, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        del ws
        return dt, info

    for w in range(args.warmup):
        log(f"warmup solve {w}")
        dt, info = run_solve(sap_prec, 0)
        log(f"  {dt:.2f}s, {info['iterations']} iterations, status {info['status']}")
    torch.cuda.synchronize()
    times, infos = [], []
    t_start = time.perf_counter()
    for k in range(args.steps):
        dt, info = run_solve(sap_prec, args.profile)
        times.append(dt)
        infos.append(info)
        log(f"step {k}: {dt:.3f}s, {info['iterations']} iterations, max true residual "
            f"{info['true_res'].max():.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ok = all(i["status"] == 0 and np.all(i["true_res"] <= cfg.tol) for i in infos)

    def rel_diff(Xa, Xb):
        """max over columns of ||Xa - Xb|| / ||Xb|| (two solutions of the same system)."""
        return float((torch.linalg.vector_norm(Xa - Xb, dim=0) / torch.linalg.vector_norm(Xb, dim=0)).max())
    X_main = Xd.clone() if not args.no_fp64_solve else None

    # the other SAP storage precision, once, for comparison
    other = None
    if not args.no_fp64_solve:
        oprec = B.FP16S if sap_prec == B.FP32 else B.FP32
        oname = "fp16s" if oprec == B.FP16S else "fp32"
        log(f"{oname}-SAP solve")
        dto, io = run_solve(oprec, 0)
        X_other = Xd.clone()
        other = {"sap_prec": oname, "seconds": dto, "tts_per_rhs_s": dto / L, "iterations": io["iterations"],
                 "max_true_res": float(io["true_res"].max()), "status": io["status"]}
        log(f"  {dto:.2f}s, {io['iterations']} iterations, max true residual {io['true_res'].max():.2e}")

    fp64 = None
    if not args.no_fp64_solve:
        log("all-FP64 solve")
        dt64, i64 = run_solve(B.FP64, 0)
        fp64 = {"seconds": dt64, "tts_per_rhs_s": dt64 / L, "iterations": i64["iterations"],
                "max_true_res": float(i64["true_res"].max()), "status": i64["status"]}
        log(f"  {dt64:.2f}s, {i64['iterations']} iterations")
        # how far the mixed-precision solutions lie from the all-FP64 one
        X64 = Xd.clone()
        fp64["max_rel_diff_of_main_solution"] = rel_diff(X_main, X64)
        if other is not None:
            other["max_rel_diff_vs_fp64_solution"] = rel_diff(X_other, X64)
            del X_other
        del X_main

    # the paper's own domain solver (SSOR, N_SSOR = 1, omega = 1.26), once, for comparison
    ssor_alt = None
    if not args.no_fp64_solve and args.domain_solver == "mr":
        log("SSOR-domain SAP solve")
        args.domain_solver = "ssor"
        dts, isr = run_solve(sap_prec, 0)
        args.domain_solver = "mr"
        ssor_alt = {"seconds": dts, "tts_per_rhs_s": dts / L, "iterations": isr["iterations"],
                    "max_true_res": float(isr["true_res"].max()), "status": isr["status"],
                    "nssor": args.nssor, "omega": args.ssor_omega,
                    "max_rel_diff_vs_fp64_solution": rel_diff(Xd, X64)}
        log(f"  {dts:.2f}s, {isr['iterations']} iterations, max true residual {isr['true_res'].max():.2e}")

    # ------------------------------------------------------------ accounting
    it = infos[-1]["iterations"]
    Vh = V // 2
    n_outer = infos[-1]["n_dslash_outer"]
    n_sap = infos[-1]["n_sap"]
    # stencil site.RHS work per solve: outer operator, SAP residual (half
    # lattice per colour) and MR domain operator (half lattice per step)
    if args.domain_solver == "ssor":
        per_sap = cfg.ncy * 2 * (1 + (2 + 2 * args.nssor) / 2) * Vh * L   # a sweep applies 4 of the 8 hops
    else:
        per_sap = cfg.ncy * 2 * (1 + cfg.nmr) * Vh * L
    stencil_work = n_outer * V * L + n_sap * per_sap
    step_s = wall / args.steps
    value = stencil_work / step_s
    km = infos[-1]["kernel_ms"]
    kl = infos[-1]["kernel_launches"]
    dominant = max(("dslash64", "mr_dslash", "mr_update", "sap_resid", "ssor"), key=lambda c: km[c])
    roof = None
    if args.profile and kl[dominant] > 0:
        # the SAP setting in force: tiled MR stencil, psi formed once
        sset = tuning.get(args.sap_prec, {}).get("sap", {}).get("setting", [])
        once = len(sset) > 7 and sset[7] == 1
        tiled = len(sset) > 6 and sset[6] >= 1
        byl = algorithmic_bytes(dominant, L, dims, cfg.block, cfg.ncy, cfg.nmr, args.sap_prec, args.nssor,
                                bool(args.csw), once, tiled)
        avg_ms = km[dominant] / kl[dominant]
        ach = byl / (avg_ms * 1e-3) / 1e9
        traffic = measured_traffic(dominant, dims, L, args.sap_prec, bool(args.csw))
        roof = {"kernel": dominant, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                "traffic_over_algorithmic": round(traffic / byl, 3) if traffic else None,
                "bytes_per_launch": byl, "avg_launch_ms": avg_ms, "launches": kl[dominant],
                "sap_tiled": tiled, "sap_psi_once": once,
                "class_ms": {k: round(v, 3) for k, v in km.items()}}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(cfg, L)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "site·RHS/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if args.sap_prec == "fp32" else "f64+f32 (fp16 storage)",
        "data": "synthetic",
        "config": {"workload": f"{'x'.join(map(str, dims))} "
                               + (f"clover-Wilson (c_sw={args.csw}, Jacobi preconditioned)" if args.csw else "Wilson-Dirac")
                               + f", L={L} point sources, "
                               f"SAP 8^4 domains ncy={cfg.ncy} "
                               + (f"nmr={cfg.nmr}" if args.domain_solver == "mr" else
                                  f"SSOR N_SSOR={args.nssor} omega={args.ssor_omega}")
                               + f", {args.sap_prec.upper()} SAP, "
                               f"tol {cfg.tol:g}",
                   "lattice": list(dims), "L": L, "kappa": cfg.kappa, "eps": cfg.eps,
                   "parallelism": "single GPU"},
        "converged": ok,
        "iterations": it,
        "tts_per_rhs_s": {"mixed": step_s / L, "fp64": fp64["tts_per_rhs_s"] if fp64 else None,
                          "fp64_over_mixed": (fp64["tts_per_rhs_s"] / (step_s / L)) if fp64 else None},
        "fp64_solve": fp64,
        "other_sap_prec_solve": other,
        "ssor_domain_solve": ssor_alt,
        "max_true_res": float(max(i["true_res"].max() for i in infos)),
        "dslash": dslash,
        "tuning": tuning,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    B.mbbs_lattice_destroy(lat)


def sweep_main(args):
    """The paper's Table 1 experiment on the 32^3x64 system: the 12 spin-colour
    point sources are solved in 12/L blocks of L consecutive components, for
    L = 1, 2, 3, 4, 6, 12.  Per L: the stand-alone operator (FP64, FP32,
    FP16 storage, tuned for that L), and the summed time, iterations and
    outer operator applications (per vector) over the blocks for the mixed
    solve (FP32 SAP, MR domains), the all-FP64 solve, and the mixed solve with
    SSOR domains (the paper's domain solver)."""
    import torch
    from paper_1104_0737_amd import autotune
    from paper_1104_0737_amd import binding as B
    from paper_1104_0737_amd import configs, model
    dims = tuple(int(x) for x in args.dims.split(","))
    cfg0 = configs.c4(L=1)
    cfg0.dims = dims
    V = int(np.prod(dims))
    N = 12 * V
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    log(f"generating links for {dims}")
    Ud = torch.from_numpy(cfg0.gauge()).to(dev)
    lat = B.mbbs_lattice_create(dims, cfg0.block, Ud, cfg0.kappa, cfg0.phases, stream=stream)
    del Ud
    site = cfg0.src_site()
    rows = []
    for L in (1, 2, 3, 4, 6, 12):
        row = {"L": L, "blocks": 12 // L, "dslash": {}}
        for prec, name in ((B.FP64, "fp64"), (B.FP32, "fp32"), (B.FP16S, "fp16s")):
            best, times = autotune.tune_operator(lat, V, L, prec, stream=stream)
            ms = times[best]
            by = model.dslash_bytes_per_site(L, name) * V
            row["dslash"][name] = {"ms": ms, "site_rhs_per_s": V * L / (ms * 1e-3),
                                   "algo_GBps": by / (ms * 1e-3) / 1e9, "setting": list(best)}
            if prec != B.FP64:
                autotune.tune_sap(lat, V, L, prec, times, stream=stream)
        torch.cuda.empty_cache()
        for key, sap_prec, dsolver in (("mixed_mr", B.FP32, 0), ("fp64_mr", B.FP64, 0), ("mixed_ssor", B.FP32, 1)):
            p = B.mbbs_solve_params_default(tol=1e-10, sap_prec=sap_prec, ncy=cfg0.ncy, nmr=cfg0.nmr,
                                            domain_solver=dsolver)
            ws = torch.empty(B.mbbs_solve_workspace_size(lat, L, p), dtype=torch.uint8, device=dev)
            tot, its, mvm, worst, ok = 0.0, [], 0, 0.0, True
            for blk in range(12 // L):
                Bd = torch.zeros((N, L), dtype=torch.complex128, device=dev)
                for j in range(L):
                    Bd[12 * site + blk * L + j, j] = 1.0
                Xd = torch.empty_like(Bd)
                torch.cuda.synchronize()
                t = time.perf_counter()
                info = B.mbbs_solve(lat, L, Bd, Xd, p, ws, stream=stream)
                torch.cuda.synchronize()
                tot += time.perf_counter() - t
                its.append(info["iterations"])
                mvm += info["n_dslash_outer"] * L
                worst = max(worst, float(info["true_res"].max()))
                ok = ok and info["status"] == 0
            row[key] = {"seconds": tot, "tts_per_rhs_s": tot / 12, "iterations": its, "outer_mvm": mvm,
                        "max_true_res": worst, "converged": ok}
            log(f"L={L:2d} {key:10s}: {tot:6.2f} s for 12 RHS, iterations {its}, max true res {worst:.1e}")
            del ws
            torch.cuda.empty_cache()
        rows.append(row)
    base = {k: rows[0][k]["seconds"] for k in ("mixed_mr", "fp64_mr", "mixed_ssor")}
    for r in rows:
        r["gain_vs_L1"] = {k: base[k] / r[k]["seconds"] for k in base}
    print(json.dumps({"sweep": rows, "workload": f"{'x'.join(map(str, dims))} Wilson, 12 point sources "
                      "in 12/L blocks, SAP 8^4 ncy=4 (MR nmr=4 or SSOR N=1 omega=1.26), tol 1e-10"}), flush=True)
    B.mbbs_lattice_destroy(lat)


def batched_main(args):
    """Batched form: 16 x 8^4 (L=4), 16 x 12^4 (L=6), 16 x 16^3x32 (L=12) systems,
    seeded links with eps ~ U[0.15, 0.3] and kappa ~ U[0.11, 0.123], half Z2 and
    half point sources, FP32 SAP, tolerance 1e-10 per column.  One step solves
    all 48 together: each size group is one batch handle whose 16 systems share
    every launch (fused), the three groups run concurrently in one batched call
    with graph_iters iterations per captured HIP graph.  Beside it: the same
    48 systems as separate handles in one batched call (concurrent but not
    fused), and one after another."""
    import torch
    from paper_1104_0737_amd import binding as B
    from paper_1104_0737_amd import configs
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    torch.cuda.set_stream(stream)
    systems = configs.c5_systems()
    groups = [systems[16 * g:16 * g + 16] for g in range(3)]
    log("generating 48 systems")
    singles, batches, Bs_single, Bs_group, Ls = [], [], [], [], []
    for grp in groups:
        Ud = []
        for s in grp:
            U = torch.from_numpy(configs.c5_gauge(s)).to(dev)
            Ud.append(U)
            singles.append(B.mbbs_lattice_create(s.dims, s.block, U, s.kappa, s.phases, stream=stream))
            Bs_single.append(torch.from_numpy(configs.c5_sources(s)).to(dev))
        s0 = grp[0]
        batches.append(B.mbbs_lattice_create_batch(s0.dims, s0.block, Ud, [s.kappa for s in grp], s0.phases,
                                                   stream=stream))
        Bs_group.append(torch.cat(Bs_single[-16:]))
        Ls.append(s0.L)
        del Ud
    torch.cuda.empty_cache()
    # launch settings: tuned on each batch handle, applied to its systems' single handles too
    tuned = {}
    if not args.no_tune:
        from paper_1104_0737_amd import autotune
        for g, (grp, bh) in enumerate(zip(groups, batches)):
            V = 16 * grp[0].V
            st = {}
            for prec in (B.FP64, B.FP32):
                best, times = autotune.tune_operator(bh, V, grp[0].L, prec, stream=stream)
                if prec != B.FP64:
                    best, _ = autotune.tune_sap(bh, V, grp[0].L, prec, times, stream=stream)
                st[prec] = best
                for lat in singles[16 * g:16 * g + 16]:
                    autotune.apply(lat, prec, best)
            tuned[(grp[0].dims, grp[0].L)] = st
            log(f"tuned {'x'.join(map(str, grp[0].dims))} L={grp[0].L}: FP64 {st[B.FP64]}, FP32 SAP {st[B.FP32]}")
        torch.cuda.empty_cache()
    params = [B.mbbs_solve_params_default(tol=1e-10, sap_prec=B.FP32, graph_iters=args.graph_iters) for _ in batches]
    ws = torch.empty(B.mbbs_solve_batched_workspace_size(batches, Ls, params), dtype=torch.uint8, device=dev)
    Xs_group = [torch.empty_like(b) for b in Bs_group]
    rhs = sum(16 * L for L in Ls)

    def run_fused():
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc, infos = B.mbbs_solve_batched(batches, Ls, Bs_group, Xs_group, params, ws, stream=stream)
        torch.cuda.synchronize()
        return time.perf_counter() - t, rc, infos

    for w in range(args.warmup):
        dt, rc, _ = run_fused()
        log(f"warmup fused batched: {dt:.3f}s rc {rc}")
    times, infos = [], None
    for k in range(args.steps):
        dt, rc, infos = run_fused()
        times.append(dt)
        log(f"step {k}: {dt:.3f}s rc {rc}")
    del ws
    torch.cuda.empty_cache()
    # the same 48 systems as separate handles in one batched call (concurrent, not fused)
    Ls48 = [s.L for s in systems]
    p48 = [B.mbbs_solve_params_default(tol=1e-10, sap_prec=B.FP32, graph_iters=args.graph_iters) for _ in systems]
    ws48 = torch.empty(B.mbbs_solve_batched_workspace_size(singles, Ls48, p48), dtype=torch.uint8, device=dev)
    Xs48 = [torch.empty_like(b) for b in Bs_single]
    B.mbbs_solve_batched(singles, Ls48, Bs_single, Xs48, p48, ws48, stream=stream)
    torch.cuda.synchronize()
    t = time.perf_counter()
    rc48, infos48 = B.mbbs_solve_batched(singles, Ls48, Bs_single, Xs48, p48, ws48, stream=stream)
    torch.cuda.synchronize()
    unfused = time.perf_counter() - t
    del ws48
    torch.cuda.empty_cache()
    log(f"separate handles, one batched call: {unfused:.3f}s rc {rc48}")
    # one after another (no graphs)
    torch.cuda.synchronize()
    t = time.perf_counter()
    seq_ok = True
    for lat, L, b, x in zip(singles, Ls48, Bs_single, Xs48):
        p = B.mbbs_solve_params_default(tol=1e-10, sap_prec=B.FP32)
        w1 = torch.empty(B.mbbs_solve_workspace_size(lat, L, p), dtype=torch.uint8, device=dev)
        info = B.mbbs_solve(lat, L, b, x, p, w1, stream=stream)
        seq_ok = seq_ok and info["status"] == 0
    torch.cuda.synchronize()
    seq = time.perf_counter() - t
    log(f"one by one: {seq:.3f}s")
    step_s = sum(times) / len(times)
    ok = all(i["status"] == 0 for i in infos)
    max_true = max(float(np.max(i["true_res"])) for i in infos)
    groups_it = {}
    for s, i in zip(systems, infos):
        groups_it.setdefault("x".join(map(str, s.dims)), []).append(i["iterations"])
    out = {"metric": "batched solve, RHS/s (48 systems, 352 RHS, FP32 SAP, tol 1e-10)", "value": rhs / step_s,
           "unit": "RHS/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_s * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32",
           "data": "synthetic", "converged": ok, "max_true_res": max_true,
           "separate_handles_s": unfused, "separate_handles_all_converged": rc48 == 0,
           "sequential_s": seq, "sequential_all_converged": seq_ok,
           "fused_over_sequential": seq / step_s, "fused_over_separate_handles": unfused / step_s,
           "iterations": {g: [min(v), max(v)] for g, v in groups_it.items()},
           "tuning": {f"{'x'.join(map(str, k[0]))} L={k[1]}": {str(p): list(v) for p, v in st.items()}
                      for k, st in tuned.items()},
           "config": {"workload": "16 x 8^4 L=4 + 16 x 12^4 L=6 + 16 x 16^3x32 L=12, SAP 4^4/6^4/8^4, "
                                  f"three batch handles (16 systems fused per launch), graph_iters={args.graph_iters}",
                      "parallelism": "single GPU"}}
    print(json.dumps(out), flush=True)
    for lat in singles + batches:
        B.mbbs_lattice_destroy(lat)


def cpu_baseline(cfg, L):
    """The oracle, untuned, on bounded samples of the workload, on the host's
    cores with BLAS held to one thread (numpy's elementwise work is
    single-threaded anyway):
    - its operator on a 32^3 x 4 slab of the lattice (the same per-site work,
      periodic in its own t extent) at the benchmark's L (the headline value)
      and at L = 1;
    - its full solve (Alg. 1, FP64, SAP with MR domains, every step in the
      oracle) of the small 8^4 system (L = 4 point sources, tol 1e-12), for a
      time to solution per right-hand side."""
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import dirac, krylov, sap
    from paper_1104_0737_amd import configs, inputs
    dims = (cfg.dims[0], cfg.dims[1], cfg.dims[2], 4)
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, cfg.eps, 99)

    def op_rate(Lc, budget):
        X = inputs.gaussian_block(V, Lc, 98)
        t = time.perf_counter()
        reps = 0
        while True:
            dirac.apply_D(U, cfg.kappa, cfg.phases, X, dims)
            reps += 1
            if time.perf_counter() - t > budget:
                break
        dt = (time.perf_counter() - t) / reps
        return V * Lc / dt, reps, dt

    with threadpool_limits(limits=1):
        blas = sorted({(i["internal_api"], i["num_threads"]) for i in threadpool_info()})
        rate, reps, dt = op_rate(L, 10.0)
        rate1, reps1, dt1 = op_rate(1, 4.0)
        c1 = configs.c1()
        U1, B1 = c1.gauge(), c1.sources()
        dom = sap.Domains(c1.dims, c1.block)
        A = lambda X: dirac.apply_D(U1, c1.kappa, c1.phases, X, c1.dims).reshape(12 * c1.V, -1)
        M = lambda X: sap.sap(U1, c1.kappa, c1.phases, dom, X, c1.ncy, c1.nmr).reshape(12 * c1.V, -1)
        t = time.perf_counter()
        res = krylov.block_bicgstab(A, M, B1, c1.tol, maxiter=100)
        ts = time.perf_counter() - t
    return {"value": rate, "unit": "site·RHS/s", "cores": 1, "kind": "oracle",
            "operator_L1_site_rhs_per_s": rate1,
            "solve": {"workload": f"{'x'.join(map(str, c1.dims))}, L={c1.L} point sources, kappa={c1.kappa}, "
                                  f"SAP {'x'.join(map(str, c1.block))} ncy={c1.ncy} nmr={c1.nmr}, FP64, tol {c1.tol:g}",
                      "seconds": ts, "iterations": res.iterations, "converged": res.converged,
                      "tts_per_rhs_s": ts / c1.L},
            "blas_threads": [list(b) for b in blas],
            "sample": f"oracle Wilson-Dirac (numpy, FP64) on a {'x'.join(map(str, dims))} slab: L={L} "
                      f"{reps} application(s) of {dt:.2f}s, L=1 {reps1} of {dt1:.2f}s; oracle solve of the "
                      f"{'x'.join(map(str, c1.dims))} system {ts:.1f}s; {len(os.sched_getaffinity(0))} host "
                      "cores visible, BLAS limited to 1 thread"}


if __name__ == "__main__":
    main()
