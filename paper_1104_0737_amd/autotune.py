"""Autotuner for the stencil kernels' launch shape.

For a lattice handle, L and a precision, time the operator over the
candidate settings (column-group width, threads per block, split-wave hop
groups, paired hops, nontemporal output stores, columns per thread, LDS-tiled
kernels) and keep the fastest on the handle.  The SAP kernels of a precision
share these settings; `tune_sap` then picks between the best split, the best
one-thread-per-site and the best tiled shape by timing the preconditioner
itself.  The split shapes and the number of columns per thread change the
order in which the hops are summed, and the MR domain sums follow the block
or tile shape; every other setting leaves the operator's result bits alone.

A setting is (group, threads, split, pair, nt[, columns per thread[, tiled[,
psi once[, columns per tiled workgroup]]]]); psi once selects the MR domain
solve that forms psi once per domain solve (a SAP-only choice).
"""

from __future__ import annotations

import itertools

from . import binding as B


def _cmax(prec):
    return 1 if prec == B.FP64 else 2


def candidates(L, prec):
    """(group columns, threads per block, split) settings: the classic kernel
    over column groups and block sizes, then the split-wave kernels."""
    c = next(c for c in range(_cmax(prec), 0, -1) if L % c == 0)
    groups = [g for g in range(c, L + 1, c) if L % g == 0]
    threads = (64, 128, 192, 256)
    classic = [(g, t, 0) for g, t in itertools.product(groups, threads)]
    return classic + [(L, 256, 2), (L, 256, 4)]


def operator_candidates(L, prec):
    """(group, threads, split, pair, nt[, columns per thread]) settings tried
    by tune_operator: all L columns or half of them per group, three block
    sizes, paired hops and nontemporal stores on or off, the other number of
    columns per thread, and the split-wave kernels."""
    c = next(c for c in range(_cmax(prec), 0, -1) if L % c == 0)
    groups = [L] + ([L // 2] if L % 2 == 0 and (L // 2) % c == 0 else [])
    out = [(g, t, 0, pr, nt) for g in groups for t in (128, 192, 256) for pr in (0, 1) for nt in (0, 1)]
    # the other number of columns per thread (FP64 automatic 1, else 2)
    other = 2 if prec == B.FP64 else 1
    if L % other == 0:
        out += [(L, t, 0, 0, nt, other) for t in (128, 256) for nt in (0, 1)]
    out += [(L, 256, sp, 0, nt) for sp in (2, 4) for nt in (0, 1)]
    # the LDS-tiled kernels (where a tile shape fits), whole-LDS and half-LDS
    # tiles, all columns or half of them per workgroup
    out += [(L, 256, 0, 0, nt, 0, tl) for tl in (1, 3) for nt in (0, 1)]
    if L % (2 * c) == 0:
        out += [(L, 256, 0, 0, nt, 0, tl, 0, L // 2) for tl in (1, 3) for nt in (0, 1)]
    return out


def _full(setting):
    """The setting with every optional element present (defaults 0)."""
    return tuple(setting) + (0,) * (9 - len(setting))


def _tiled(setting):
    return len(setting) > 6 and setting[6] >= 1


def apply(lat, prec, setting):
    g, t, sp, pr, nt = setting[:5]
    ch = setting[5] if len(setting) > 5 else 0
    B.mbbs_lattice_tune(lat, B.TUNE_TILE[prec], setting[6] if _tiled(setting) else 0)
    B.mbbs_lattice_tune(lat, B.TUNE_MR_ONCE[prec], setting[7] if len(setting) > 7 else 0)
    B.mbbs_lattice_tune(lat, B.TUNE_TILE_COLS[prec], setting[8] if len(setting) > 8 else 0)
    B.mbbs_lattice_tune(lat, B.TUNE_CHUNK[prec], ch)
    B.mbbs_lattice_tune(lat, B.TUNE_GROUP[prec], g)
    B.mbbs_lattice_tune(lat, B.TUNE_BLOCK_THREADS_PREC[prec], t)
    B.mbbs_lattice_tune(lat, B.TUNE_SPLIT[prec], sp)
    B.mbbs_lattice_tune(lat, B.TUNE_HOP_PAIR[prec], pr)
    B.mbbs_lattice_tune(lat, B.TUNE_NT_STORE[prec], nt)


def tune_operator(lat, V, L, prec, stream=None, reps=3):
    """Return (best setting, {setting: ms}) and apply the best."""
    import torch
    dev = torch.device("cuda")
    N = 12 * V
    if prec == B.FP64:
        X = torch.zeros((N, L), dtype=torch.complex128, device=dev)
        Xs = Ys = None
    else:
        dt = torch.float32 if prec == B.FP32 else torch.float16
        X = torch.zeros((N, L, 2), dtype=dt, device=dev)
        Xs = torch.ones((V, L), dtype=torch.float32, device=dev) if prec == B.FP16S else None
        Ys = torch.empty_like(Xs) if Xs is not None else None
    Y = torch.empty_like(X)
    s = stream or torch.cuda.current_stream()
    times = {}
    for setting in operator_candidates(L, prec):
        apply(lat, prec, setting)
        B.mbbs_apply_dirac_raw(lat, L, prec, X, Xs, Y, Ys, stream=s)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            B.mbbs_apply_dirac_raw(lat, L, prec, X, Xs, Y, Ys, stream=s)
        e1.record(s)
        e1.synchronize()
        times[setting] = e0.elapsed_time(e1) / reps
    best = min(times, key=times.get)
    apply(lat, prec, best)
    del X, Y, Xs, Ys
    return best, times


def sap_candidates(L, prec, op_times):
    """The SAP settings tune_sap times, from tune_operator's timings: the
    fastest split, one-thread-per-site and tiled operator settings, the tiled
    one with the MR update folded in (FP64 / FP32), with the other tile sizes
    (whole or half LDS, all or half the columns per workgroup), the tiled MR
    step under the fastest one-thread-per-site shape, each of these with psi
    formed once, and one column per thread (FP32 / FP16 storage)."""
    split = [k for k in op_times if k[2] in (2, 4)]
    classic = [k for k in op_times if k[2] not in (2, 4) and not _tiled(k)]
    tiled = [k for k in op_times if _tiled(k)]
    cands = [min(c, key=op_times.get) for c in (split, classic, tiled) if c]
    folded = prec != B.FP16S          # the folded MR update: FP64 and FP32 only
    if tiled and folded:
        # the MR update folded into the next MR step
        cands.append(tuple(min(tiled, key=op_times.get)[:6]) + (2,))
    if tiled:
        # the other tile sizes than the operator's fastest: whole or half LDS,
        # all columns or half of them per workgroup
        bt = min(tiled, key=op_times.get)
        c = next(c for c in range(_cmax(prec), 0, -1) if L % c == 0)
        halves = [L // 2] if L % (2 * c) == 0 else []
        seen = {_full(x) for x in cands}
        for tl in (1, 3):
            for lg in [0] + halves:
                v = tuple(bt[:6]) + (tl, 0) + ((lg,) if lg else ())
                if _full(v) not in seen:
                    cands.append(v)
                    seen.add(_full(v))
    if classic and tiled:
        # the SAP residual kernel in the best classic shape, the MR step tiled
        best = min(classic, key=op_times.get)
        base = tuple(best[:5]) + ((best[5] if len(best) > 5 else 0),)
        cands += [base + (1,), base + (3,)] + ([base + (2,)] if folded else [])
    # psi formed once per domain solve, on the untiled and tiled candidates
    pad = lambda c: tuple(c[:5]) + tuple(c[5:7]) + (0,) * (7 - len(c[:7]))
    cands += [pad(c) + (1,) + tuple(c[8:9]) for c in list(cands) if not (len(c) > 6 and c[6] == 2)]
    if classic and prec != B.FP64:
        # one column per thread: more waves in flight per CU for the domain kernels
        g, t, sp, pr, nt = min(classic, key=op_times.get)[:5]
        cands += [(L, tt, 0, pv, nt, 1) for tt in (128, 256) for pv in (0, 1)]
        cands += [(L, 256, 0, 1, nt, 0)]
    return cands


def tune_sap(lat, V, L, prec, op_times, stream=None, ncy=4, nmr=4, reps=2):
    """Of sap_candidates' settings keep the one under which the SAP
    preconditioner itself runs faster.  Returns (setting, {setting: ms})."""
    import torch
    cands = sap_candidates(L, prec, op_times)
    dev = torch.device("cuda")
    s = stream or torch.cuda.current_stream()
    X = torch.zeros((12 * V, L), dtype=torch.complex128, device=dev)
    X[::7] = 1.0
    Y = torch.empty_like(X)
    times = {}
    for setting in cands:
        apply(lat, prec, setting)
        # the workspace depends on the setting (the folded MR update needs more)
        ws = torch.empty(B.mbbs_sap_workspace_size(lat, L, prec), dtype=torch.uint8, device=dev)
        B.mbbs_sap_apply(lat, L, X, Y, ncy, nmr, prec, ws, stream=s)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            B.mbbs_sap_apply(lat, L, X, Y, ncy, nmr, prec, ws, stream=s)
        e1.record(s)
        e1.synchronize()
        times[setting] = e0.elapsed_time(e1) / reps
        del ws
    best = min(times, key=times.get)
    apply(lat, prec, best)
    del X, Y
    return best, times
