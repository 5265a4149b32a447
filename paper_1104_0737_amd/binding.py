"""Thin ctypes binding of libmbbs.so: the C ABI's names, argument marshalling only.

Device arrays are torch tensors on the current HIP device (complex128 for
FP64 spinor blocks and links); host arrays are numpy arrays.  Every function
raises MbbsError on a negative status.  The library must be built first
(`python -m paper_1104_0737_amd.build`); nothing here falls back to any other
implementation.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbbs.so")

FP64, FP32, FP16S = 0, 1, 2
OK, NOT_CONVERGED, EINVAL, ENOMEM, EHIP, EBREAKDOWN = 0, 1, -1, -2, -3, -4
TABLES = ("COORD", "NEIGHBOUR", "BOUNDARY", "PARITY", "EO", "DOMAIN", "COLOUR", "LOCAL",
          "DM_INDEX", "DM_SITE", "LOCAL_NB", "DM_NEIGHBOUR", "HYPERPLANE")
KERNEL_CLASSES = ("dslash64", "sap_resid", "mr_dslash", "mr_update", "convert", "gram", "update", "small", "ssor")

EXPORTS = (
    "mbbs_lattice_create", "mbbs_lattice_create_batch", "mbbs_lattice_nsys", "mbbs_lattice_destroy", "mbbs_lattice_tune", "mbbs_lattice_tile_shape",
    "mbbs_lattice_set_clover",
    "mbbs_lattice_clover_inverse", "mbbs_apply_clover_inverse", "mbbs_lattice_table_size",
    "mbbs_lattice_table",
    "mbbs_apply_dirac", "mbbs_apply_dirac_raw", "mbbs_convert_to", "mbbs_convert_from",
    "mbbs_apply_blocked", "mbbs_sap_workspace_size", "mbbs_sap_apply", "mbbs_ssor_workspace_size",
    "mbbs_sap_apply_ssor", "mbbs_apply_ssor_blocked", "mbbs_gram_workspace_size",
    "mbbs_gram", "mbbs_gram_noalloc", "mbbs_cholqr", "mbbs_lu_solve", "mbbs_solve_params_default",
    "mbbs_solve_workspace_size", "mbbs_solve", "mbbs_solve_batched_workspace_size",
    "mbbs_solve_batched", "mbbs_last_error",
)


class MbbsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mbbs error {code}: {msg}")
        self.code = code


class SolveParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxiter", ctypes.c_int), ("max_restarts", ctypes.c_int),
                ("ncy", ctypes.c_int), ("nmr", ctypes.c_int), ("sap_prec", ctypes.c_int),
                ("x0_is_guess", ctypes.c_int), ("qr_passes", ctypes.c_int), ("graph_iters", ctypes.c_int),
                ("precond", ctypes.c_int), ("memsave", ctypes.c_int), ("profile", ctypes.c_int),
                ("domain_solver", ctypes.c_int), ("nssor", ctypes.c_int), ("ssor_omega", ctypes.c_double),
                ("rtilde", ctypes.c_void_p)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int), ("restarts", ctypes.c_int),
                ("n_dslash_outer", ctypes.c_longlong), ("n_sap", ctypes.c_longlong),
                ("true_res", ctypes.POINTER(ctypes.c_double)), ("rec_res", ctypes.POINTER(ctypes.c_double)),
                ("seconds", ctypes.c_double), ("kernel_ms", ctypes.c_double * len(KERNEL_CLASSES)),
                ("kernel_launches", ctypes.c_longlong * len(KERNEL_CLASSES)),
                ("res_history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int),
                ("history_len", ctypes.c_int)]

HISTORY_CAP = 4096   # residual-history entries the library keeps


_lib = None


def lib():
    """Load libmbbs.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1104_0737_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
        sig = {
            "mbbs_lattice_create": (i, [ctypes.POINTER(i), ctypes.POINTER(i), vp, d, ctypes.POINTER(d), vp,
                                        ctypes.POINTER(vp)]),
            "mbbs_lattice_create_batch": (i, [i, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(vp),
                                              ctypes.POINTER(d), ctypes.POINTER(d), vp, ctypes.POINTER(vp)]),
            "mbbs_lattice_nsys": (i, [vp, ctypes.POINTER(i)]),
            "mbbs_lattice_destroy": (i, [vp]),
            "mbbs_lattice_tune": (i, [vp, i, i]),
            "mbbs_lattice_tile_shape": (i, [vp, i, i, ctypes.POINTER(ctypes.c_int32)]),
            "mbbs_lattice_set_clover": (i, [vp, d, vp]),
            "mbbs_lattice_clover_inverse": (i, [vp, vp, vp]),
            "mbbs_apply_clover_inverse": (i, [vp, i, vp, vp, vp]),
            "mbbs_lattice_table_size": (i, [vp, i, ctypes.POINTER(sz)]),
            "mbbs_lattice_table": (i, [vp, i, vp, sz]),
            "mbbs_apply_dirac": (i, [vp, i, vp, vp, i, vp]),
            "mbbs_apply_dirac_raw": (i, [vp, i, i, vp, vp, vp, vp, vp]),
            "mbbs_convert_to": (i, [i, sz, i, vp, vp, vp, vp]),
            "mbbs_convert_from": (i, [i, sz, i, vp, vp, vp, vp]),
            "mbbs_apply_blocked": (i, [vp, i, vp, vp, i, vp]),
            "mbbs_sap_workspace_size": (i, [vp, i, i, ctypes.POINTER(sz)]),
            "mbbs_sap_apply": (i, [vp, i, vp, vp, i, i, i, vp, sz, vp]),
            "mbbs_ssor_workspace_size": (i, [vp, i, i, ctypes.POINTER(sz)]),
            "mbbs_sap_apply_ssor": (i, [vp, i, vp, vp, i, i, d, i, vp, sz, vp]),
            "mbbs_apply_ssor_blocked": (i, [vp, i, vp, vp, i, d, i, vp, sz, vp]),
            "mbbs_gram_workspace_size": (i, [sz, i, ctypes.POINTER(sz)]),
            "mbbs_gram": (i, [sz, i, vp, vp, vp, vp, sz, vp]),
            "mbbs_gram_noalloc": (i, [sz, i, vp, vp, vp, vp]),
            "mbbs_cholqr": (i, [sz, i, vp, vp, vp, i, vp, sz, vp]),
            "mbbs_lu_solve": (i, [i, i, vp, vp, vp, vp]),
            "mbbs_solve_params_default": (None, [ctypes.POINTER(SolveParams)]),
            "mbbs_solve_workspace_size": (i, [vp, i, ctypes.POINTER(SolveParams), ctypes.POINTER(sz)]),
            "mbbs_solve": (i, [vp, i, vp, vp, ctypes.POINTER(SolveParams), vp, sz, ctypes.POINTER(SolveInfo), vp]),
            "mbbs_solve_batched_workspace_size": (i, [i, ctypes.POINTER(vp), ctypes.POINTER(i),
                                                      ctypes.POINTER(SolveParams), ctypes.POINTER(sz)]),
            "mbbs_solve_batched": (i, [i, ctypes.POINTER(vp), ctypes.POINTER(i), ctypes.POINTER(vp),
                                       ctypes.POINTER(vp), ctypes.POINTER(SolveParams), vp, sz,
                                       ctypes.POINTER(SolveInfo), vp]),
            "mbbs_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise MbbsError(rc, lib().mbbs_last_error().decode())
    return rc


def _dev(t, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("device tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _opt(t):
    return ctypes.c_void_p(0) if t is None else _dev(t)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _c128():
    import torch
    return torch.complex128


# ----------------------------------------------------------------- lattice
def mbbs_lattice_create(dims, block, U, kappa, phases, stream=None):
    """U: complex128 device tensor (V, 4, 3, 3); phases: 4 (re, im) pairs."""
    d = (ctypes.c_int * 4)(*dims)
    b = (ctypes.c_int * 4)(*block)
    ph = (ctypes.c_double * 8)(*[float(x) for p in phases for x in p])
    out = ctypes.c_void_p()
    _check(lib().mbbs_lattice_create(d, b, _dev(U, _c128()), float(kappa), ph, _stream(stream), ctypes.byref(out)))
    return out


def mbbs_lattice_create_batch(dims, block, Us, kappas, phases, stream=None):
    """A batch of len(Us) same-shape systems in one handle: Us are complex128
    device tensors (V, 4, 3, 3), kappas one value per system."""
    n = len(Us)
    if len(kappas) != n:
        raise ValueError("one kappa per system")
    d = (ctypes.c_int * 4)(*dims)
    b = (ctypes.c_int * 4)(*block)
    up = (ctypes.c_void_p * n)(*[_dev(u, _c128()).value for u in Us])
    kp = (ctypes.c_double * n)(*[float(k) for k in kappas])
    ph = (ctypes.c_double * 8)(*[float(x) for p in phases for x in p])
    out = ctypes.c_void_p()
    _check(lib().mbbs_lattice_create_batch(n, d, b, up, kp, ph, _stream(stream), ctypes.byref(out)))
    return out


def mbbs_lattice_nsys(lat):
    n = ctypes.c_int()
    _check(lib().mbbs_lattice_nsys(lat, ctypes.byref(n)))
    return n.value


def mbbs_lattice_destroy(lat):
    return _check(lib().mbbs_lattice_destroy(lat))


TUNE_GROUP = {0: 0, 1: 1, 2: 2}      # precision -> knob
TUNE_BLOCK_THREADS = 3                 # every precision
TUNE_BLOCK_THREADS_PREC = {0: 20, 1: 21, 2: 22}   # precision -> knob
TUNE_LDS_PAD_KB = 4
TUNE_SPLIT = {0: 5, 1: 6, 2: 7}      # precision -> knob
TUNE_PERSIST_BLOCKS = 8
TUNE_MR_FUSED = 9
TUNE_MR_ONCE = {0: 26, 1: 27, 2: 28}    # precision -> knob
TUNE_NT_STORE = {0: 14, 1: 15, 2: 16}   # precision -> knob
TUNE_CHUNK = {0: 17, 1: 18, 2: 19}      # precision -> knob
TUNE_HOP_PAIR = {0: 11, 1: 12, 2: 13}   # precision -> knob
TUNE_TILE = {0: 23, 1: 24, 2: 25}       # precision -> knob
TUNE_TILE_COLS = {0: 29, 1: 30, 2: 31}  # precision -> knob


def mbbs_lattice_tune(lat, knob, value):
    return _check(lib().mbbs_lattice_tune(lat, knob, value))


def mbbs_lattice_tile_shape(lat, L, prec):
    """Tile extents of the LDS-tiled kernels for (L, prec), or (0, 0, 0, 0)."""
    t = (ctypes.c_int32 * 4)()
    _check(lib().mbbs_lattice_tile_shape(lat, L, prec, t))
    return tuple(t)


def mbbs_lattice_set_clover(lat, csw, stream=None):
    return _check(lib().mbbs_lattice_set_clover(lat, ctypes.c_double(csw), _stream(stream)))


def mbbs_lattice_clover_inverse(lat, out, stream=None):
    """out: complex128 device tensor (V, 12, 12)."""
    return _check(lib().mbbs_lattice_clover_inverse(lat, _dev(out, _c128()), _stream(stream)))


def mbbs_apply_clover_inverse(lat, L, X, Y, stream=None):
    return _check(lib().mbbs_apply_clover_inverse(lat, L, _dev(X, _c128()), _dev(Y, _c128()), _stream(stream)))


def mbbs_lattice_table(lat, which):
    """Table `which` (int or name) as an int32 numpy array."""
    if isinstance(which, str):
        which = TABLES.index(which)
    n = ctypes.c_size_t()
    _check(lib().mbbs_lattice_table_size(lat, which, ctypes.byref(n)))
    out = np.empty(n.value, dtype=np.int32)
    _check(lib().mbbs_lattice_table(lat, which, out.ctypes.data_as(ctypes.c_void_p), n.value))
    return out


# ----------------------------------------------------------------- operator
def mbbs_apply_dirac(lat, L, X, Y, prec=FP64, stream=None):
    return _check(lib().mbbs_apply_dirac(lat, L, _dev(X, _c128()), _dev(Y, _c128()), prec, _stream(stream)))


def mbbs_apply_dirac_raw(lat, L, prec, X, Xs, Y, Ys, stream=None):
    return _check(lib().mbbs_apply_dirac_raw(lat, L, prec, _dev(X), _opt(Xs), _dev(Y), _opt(Ys), _stream(stream)))


def mbbs_convert_to(prec, nsites, L, X, Y, Ys=None, stream=None):
    return _check(lib().mbbs_convert_to(prec, nsites, L, _dev(X, _c128()), _dev(Y), _opt(Ys), _stream(stream)))


def mbbs_convert_from(prec, nsites, L, X, Xs, Y, stream=None):
    return _check(lib().mbbs_convert_from(prec, nsites, L, _dev(X), _opt(Xs), _dev(Y, _c128()), _stream(stream)))


def mbbs_apply_blocked(lat, L, X, Y, prec=FP64, stream=None):
    return _check(lib().mbbs_apply_blocked(lat, L, _dev(X, _c128()), _dev(Y, _c128()), prec, _stream(stream)))


def mbbs_sap_workspace_size(lat, L, prec):
    n = ctypes.c_size_t()
    _check(lib().mbbs_sap_workspace_size(lat, L, prec, ctypes.byref(n)))
    return n.value


def mbbs_sap_apply(lat, L, X, Y, ncy, nmr, prec, ws, stream=None):
    return _check(lib().mbbs_sap_apply(lat, L, _dev(X, _c128()), _dev(Y, _c128()), ncy, nmr, prec, _dev(ws),
                                       ws.numel() * ws.element_size(), _stream(stream)))


# ----------------------------------------------------------------- block LA
def mbbs_ssor_workspace_size(lat, L, prec):
    n = ctypes.c_size_t()
    _check(lib().mbbs_ssor_workspace_size(lat, L, prec, ctypes.byref(n)))
    return n.value


def mbbs_sap_apply_ssor(lat, L, X, Y, ncy, nssor, omega, prec, ws, stream=None):
    return _check(lib().mbbs_sap_apply_ssor(lat, L, _dev(X, _c128()), _dev(Y, _c128()), ncy, nssor,
                                            ctypes.c_double(omega), prec, _dev(ws), ws.numel() * ws.element_size(),
                                            _stream(stream)))


def mbbs_apply_ssor_blocked(lat, L, X, Y, nssor, omega, prec, ws, stream=None):
    return _check(lib().mbbs_apply_ssor_blocked(lat, L, _dev(X, _c128()), _dev(Y, _c128()), nssor,
                                                ctypes.c_double(omega), prec, _dev(ws),
                                                ws.numel() * ws.element_size(), _stream(stream)))


def mbbs_gram_workspace_size(N, L):
    n = ctypes.c_size_t()
    _check(lib().mbbs_gram_workspace_size(N, L, ctypes.byref(n)))
    return n.value


def mbbs_gram(N, L, X, Y, G, ws, stream=None):
    return _check(lib().mbbs_gram(N, L, _dev(X, _c128()), _dev(Y, _c128()), _dev(G, _c128()), _dev(ws),
                                  ws.numel() * ws.element_size(), _stream(stream)))


def mbbs_gram_noalloc(N, L, X, Y, G, stream=None):
    return _check(lib().mbbs_gram_noalloc(N, L, _dev(X, _c128()), _dev(Y, _c128()), _dev(G, _c128()),
                                          _stream(stream)))


def mbbs_cholqr(N, L, P, Q, gamma, passes, ws, stream=None):
    return _check(lib().mbbs_cholqr(N, L, _dev(P, _c128()), _dev(Q, _c128()), _dev(gamma, _c128()), passes,
                                    _dev(ws), ws.numel() * ws.element_size(), _stream(stream)))


def mbbs_lu_solve(L, m, G, R, X, stream=None):
    return _check(lib().mbbs_lu_solve(L, m, _dev(G, _c128()), _dev(R, _c128()), _dev(X, _c128()),
                                      _stream(stream)))


# ----------------------------------------------------------------- solver
def mbbs_solve_params_default(**overrides):
    """Default parameters with overrides; rtilde may be a complex128 device
    tensor (N, L) holding R~ (the caller keeps it alive during the solve)."""
    p = SolveParams()
    lib().mbbs_solve_params_default(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        if k == "rtilde":
            v = None if v is None else _dev(v, _c128()).value
        setattr(p, k, v)
    return p


def mbbs_solve_workspace_size(lat, L, params):
    n = ctypes.c_size_t()
    _check(lib().mbbs_solve_workspace_size(lat, L, ctypes.byref(params), ctypes.byref(n)))
    return n.value


def _attach(info, L):
    tr = (ctypes.c_double * L)()
    rr = (ctypes.c_double * L)()
    hist = (ctypes.c_double * HISTORY_CAP)()
    info.true_res = ctypes.cast(tr, ctypes.POINTER(ctypes.c_double))
    info.rec_res = ctypes.cast(rr, ctypes.POINTER(ctypes.c_double))
    info.res_history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
    info.history_cap = HISTORY_CAP
    return tr, rr, hist


def _info(L):
    info = SolveInfo()
    return (info, *_attach(info, L))


def _info_dict(info, tr, rr, hist, rc):
    return {"status": rc, "iterations": info.iterations, "restarts": info.restarts,
            "n_dslash_outer": info.n_dslash_outer, "n_sap": info.n_sap,
            "true_res": np.array(tr[:]), "rec_res": np.array(rr[:]), "seconds": info.seconds,
            "kernel_ms": dict(zip(KERNEL_CLASSES, info.kernel_ms[:])),
            "kernel_launches": dict(zip(KERNEL_CLASSES, info.kernel_launches[:])),
            "history": np.array(hist[:max(0, info.history_len)])}


def mbbs_solve(lat, L, B, X, params, ws, stream=None):
    """Single-system handle: returns a dict (status, iterations, restarts,
    residuals, timings, history).  Batch handle (B, X the stacked blocks):
    returns (worst status, [dict per system]) and raises only when the call
    failed before any system was solved."""
    ns = mbbs_lattice_nsys(lat)
    infos = (SolveInfo * ns)()
    keep = [_attach(infos[k], L) for k in range(ns)]
    unset = 99                          # not an mbbs status: marks a record the call never filled
    for k in range(ns):
        infos[k].status = unset
    rc = lib().mbbs_solve(lat, L, _dev(B, _c128()), _dev(X, _c128()), ctypes.byref(params), _dev(ws),
                          ws.numel() * ws.element_size(), infos, _stream(stream))
    if ns == 1:
        _check(rc)
        return _info_dict(infos[0], *keep[0], rc)
    if rc < 0 and all(infos[k].status in (unset, rc) for k in range(ns)):
        _check(rc)
    return rc, [_info_dict(infos[k], *keep[k], infos[k].status) for k in range(ns)]


def mbbs_solve_batched_workspace_size(lats, Ls, params):
    n = len(lats)
    la = (ctypes.c_void_p * n)(*[x.value for x in lats])
    Li = (ctypes.c_int * n)(*Ls)
    pa = (SolveParams * n)(*params)
    out = ctypes.c_size_t()
    _check(lib().mbbs_solve_batched_workspace_size(n, la, Li, pa, ctypes.byref(out)))
    return out.value


def mbbs_solve_batched(lats, Ls, Bs, Xs, params, ws, stream=None):
    """Returns (worst status, [info dict per system]).  Raises MbbsError only
    when the call fails before any system is solved (arguments, workspace)."""
    n = len(lats)
    la = (ctypes.c_void_p * n)(*[x.value for x in lats])
    Li = (ctypes.c_int * n)(*Ls)
    Bp = (ctypes.c_void_p * n)(*[_dev(b, _c128()).value for b in Bs])
    Xp = (ctypes.c_void_p * n)(*[_dev(x, _c128()).value for x in Xs])
    pa = (SolveParams * n)(*params)
    nsys = [mbbs_lattice_nsys(x) for x in lats]
    sysL = [L for L, m in zip(Ls, nsys) for _ in range(m)]
    ntot = len(sysL)
    infos = (SolveInfo * ntot)()
    keep = [_attach(infos[k], sysL[k]) for k in range(ntot)]
    unset = 99                          # not an mbbs status: marks a record the call never filled
    for k in range(ntot):
        infos[k].status = unset
    rc = lib().mbbs_solve_batched(n, la, Li, Bp, Xp, pa, _dev(ws), ws.numel() * ws.element_size(), infos,
                                  _stream(stream))
    if rc < 0 and all(infos[k].status == unset for k in range(ntot)):
        _check(rc)                      # the call failed before solving anything
    # per-system failures: the return value is the worst status, each record has its own
    return rc, [_info_dict(infos[k], *keep[k], infos[k].status) for k in range(ntot)]


def mbbs_last_error():
    return lib().mbbs_last_error().decode()
