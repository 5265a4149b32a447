"""The C ABI's host paths under the address and undefined-behaviour
sanitizers (no GPU): the library's host code is rebuilt with both (device
code left out), the sanitizer runtime is preloaded into a fresh Python, and
every entry point is driven through its argument checks, defaults and size
computations.  Any sanitizer report fails the test."""

import os
import subprocess
import sys

import pytest

from paper_1104_0737_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
import ctypes, sys
sys.path.insert(0, ROOT)
from paper_1104_0737_amd import binding as B
B.LIB_PATH = SAN_LIB
lib = B.lib()
vp, ci = ctypes.c_void_p, ctypes.c_int
fake = vp(0x1000)          # never dereferenced: every call below fails its checks first
out = vp()
ph = (ctypes.c_double * 8)(1, 0, 1, 0, 1, 0, -1, 0)
bad_ph = (ctypes.c_double * 8)(1, 0, 1, 0, 1, 0, -2, 0)
sz = ctypes.c_size_t()
dims = lambda *d: (ci * 4)(*d)
calls = [
    lambda: lib.mbbs_lattice_create(dims(4, 4, 4, 5), dims(2, 2, 2, 5), fake, 0.1, ph, None, ctypes.byref(out)),
    lambda: lib.mbbs_lattice_create(dims(4, 4, 4, 6), dims(2, 2, 2, 2), fake, 0.1, ph, None, ctypes.byref(out)),
    lambda: lib.mbbs_lattice_create(dims(4, 4, 4, 8), dims(2, 2, 2, 3), fake, 0.1, ph, None, ctypes.byref(out)),
    lambda: lib.mbbs_lattice_create(dims(4, 4, 4, 4), dims(2, 2, 2, 2), fake, 0.1, bad_ph, None, ctypes.byref(out)),
    lambda: lib.mbbs_lattice_create(dims(0, 4, 4, 4), dims(2, 2, 2, 2), fake, 0.1, ph, None, ctypes.byref(out)),
    lambda: lib.mbbs_lattice_create(dims(4, 4, 4, 4), dims(2, 2, 2, 2), None, 0.1, ph, None, ctypes.byref(out)),
    lambda: lib.mbbs_lattice_create_batch(0, dims(4, 4, 4, 4), dims(2, 2, 2, 2), None, None, ph, None,
                                          ctypes.byref(out)),
    lambda: lib.mbbs_apply_dirac(fake, 0, vp(32), vp(64), 0, None),
    lambda: lib.mbbs_apply_dirac(fake, 257, vp(32), vp(64), 0, None),
    lambda: lib.mbbs_apply_dirac(fake, 4, vp(32), vp(32), 0, None),
    lambda: lib.mbbs_apply_dirac(fake, 4, vp(32), vp(64), 7, None),
    lambda: lib.mbbs_apply_blocked(None, 4, vp(32), vp(64), 0, None),
    lambda: lib.mbbs_apply_dirac_raw(fake, 4, 2, vp(32), None, vp(64), None, None),
    lambda: lib.mbbs_convert_to(2, 16, 4, vp(32), vp(64), None, None),
    lambda: lib.mbbs_convert_from(9, 16, 4, vp(32), None, vp(64), None),
    lambda: lib.mbbs_sap_workspace_size(None, 4, 1, ctypes.byref(sz)),
    lambda: lib.mbbs_sap_apply(fake, 65, vp(32), vp(64), 4, 4, 1, vp(96), 1 << 20, None),
    lambda: lib.mbbs_sap_apply(fake, 4, vp(32), vp(64), 0, 4, 1, vp(96), 1 << 20, None),
    lambda: lib.mbbs_ssor_workspace_size(fake, 0, 1, ctypes.byref(sz)),
    lambda: lib.mbbs_sap_apply_ssor(fake, 4, vp(32), vp(64), 4, 2, ctypes.c_double(1.26), 1, vp(96), 1 << 20, None),
    lambda: lib.mbbs_sap_apply_ssor(fake, 4, vp(32), vp(64), 4, 1, ctypes.c_double(2.5), 1, vp(96), 1 << 20, None),
    lambda: lib.mbbs_apply_ssor_blocked(fake, 4, vp(32), vp(32), 1, ctypes.c_double(1.0), 1, vp(96), 1 << 20, None),
    lambda: lib.mbbs_gram_workspace_size(100, 0, ctypes.byref(sz)),
    lambda: lib.mbbs_gram(100, 17, vp(32), vp(64), vp(96), vp(128), 1 << 20, None),
    lambda: lib.mbbs_gram(100, 4, vp(32), vp(64), vp(96), vp(128), 0, None),
    lambda: lib.mbbs_gram_noalloc(100, 17, vp(32), vp(64), vp(96), None),
    lambda: lib.mbbs_cholqr(100, 4, vp(32), vp(64), vp(96), 3, vp(128), 1 << 20, None),
    lambda: lib.mbbs_cholqr(100, 4, vp(32), vp(64), vp(96), 1, vp(128), 0, None),
    lambda: lib.mbbs_lu_solve(33, 1, vp(32), vp(64), vp(96), None),
    lambda: lib.mbbs_lattice_tune(None, 0, 1),
    lambda: lib.mbbs_lattice_tile_shape(None, 12, 1, None),
    lambda: lib.mbbs_lattice_set_clover(None, ctypes.c_double(1.0), None),
]
for k, f in enumerate(calls):
    rc = f()
    assert rc == B.EINVAL, (k, rc, B.mbbs_last_error())
    assert B.mbbs_last_error(), k
# defaults, sizes and the solver's own checks
p = B.mbbs_solve_params_default()
assert p.tol == 1e-10 and p.ncy == 4 and p.nmr == 4
for N, L in ((49152, 4), (12 * 4096, 12), (25165824, 16), (1, 1)):
    assert B.mbbs_gram_workspace_size(N, L) > 0
pp = B.mbbs_solve_params_default()
rc = lib.mbbs_solve_workspace_size(None, 4, ctypes.byref(pp), ctypes.byref(sz))
assert rc == B.EINVAL
for bad in (dict(tol=0.0), dict(tol=-1.0), dict(tol=float("inf")), dict(ncy=0), dict(nmr=0), dict(maxiter=-1),
            dict(sap_prec=7), dict(qr_passes=3), dict(domain_solver=2), dict(domain_solver=1, nssor=2),
            dict(domain_solver=1, ssor_omega=2.5)):
    q = B.mbbs_solve_params_default(**bad)
    rc = lib.mbbs_solve(fake, 4, vp(32), vp(64), ctypes.byref(q), vp(96), 1 << 30, None, None)
    assert rc == B.EINVAL, (bad, rc, B.mbbs_last_error())
print("host paths ok", len(calls))
'''


def test_abi_host_paths_under_sanitizers(tmp_path):
    rt = build.sanitizer_runtime()
    if not rt or not os.path.exists(rt):
        pytest.skip("no address-sanitizer runtime beside hipcc's clang")
    lib = build.build_sanitized()
    # the library is instrumented: it calls into both runtimes
    syms = subprocess.run(["nm", "-D", lib], capture_output=True, text=True).stdout
    assert "__asan_report_load" in syms and "__ubsan_handle_" in syms
    src = tmp_path / "drive.py"
    src.write_text(f"ROOT = {ROOT!r}\nSAN_LIB = {lib!r}\n" + DRIVER)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, str(src)], env=env, capture_output=True, text=True, timeout=300)
    report = r.stdout + r.stderr
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert r.returncode == 0, report[-4000:]
    assert "host paths ok" in r.stdout
