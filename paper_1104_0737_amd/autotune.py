"""Autotuner for the stencil kernels' launch shape.

For a lattice handle, L and a precision, time the operator (what the SAP
kernels of that precision share: column-group width and threads per block)
over the candidate settings and keep the fastest on the handle.  Every
setting produces bit-identical results, so the choice only affects speed.
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


def tune_operator(lat, V, L, prec, stream=None, reps=3):
    """Return (best (group, threads, split), {setting: ms}) and apply the best."""
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
    for g, t, sp in candidates(L, prec):
        B.mbbs_lattice_tune(lat, B.TUNE_GROUP[prec], g)
        B.mbbs_lattice_tune(lat, B.TUNE_BLOCK_THREADS, t)
        B.mbbs_lattice_tune(lat, B.TUNE_SPLIT[prec], sp)
        B.mbbs_apply_dirac_raw(lat, L, prec, X, Xs, Y, Ys, stream=s)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            B.mbbs_apply_dirac_raw(lat, L, prec, X, Xs, Y, Ys, stream=s)
        e1.record(s)
        e1.synchronize()
        times[(g, t, sp)] = e0.elapsed_time(e1) / reps
    best = min(times, key=times.get)
    B.mbbs_lattice_tune(lat, B.TUNE_GROUP[prec], best[0])
    B.mbbs_lattice_tune(lat, B.TUNE_BLOCK_THREADS, best[1])
    B.mbbs_lattice_tune(lat, B.TUNE_SPLIT[prec], best[2])
    del X, Y, Xs, Ys
    return best, times
