"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/mbbs.h declares, and rejects bad arguments before
touching the device."""

import ctypes
import os
import re

import pytest

from paper_1104_0737_amd import binding

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mbbs.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mbbs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_binding_exports():
    assert _declared() == sorted(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = binding.lib()
    for name in _declared():
        assert hasattr(lib, name), name
        assert isinstance(getattr(lib, name), ctypes._CFuncPtr)


def test_defaults_and_sizes_without_device():
    p = binding.mbbs_solve_params_default()
    assert p.tol == 1e-10 and p.maxiter == 1000 and p.ncy == 4 and p.nmr == 4
    assert p.sap_prec == binding.FP32 and p.precond == 1 and p.qr_passes == 1
    assert binding.mbbs_gram_workspace_size(12 * 4096, 12) > 0
    with pytest.raises(binding.MbbsError):
        binding.mbbs_gram_workspace_size(100, 0)


def test_create_validates_before_device_work():
    lib = binding.lib()
    out = ctypes.c_void_p()
    ph = (ctypes.c_double * 8)(1, 0, 1, 0, 1, 0, -1, 0)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    for dims, block in (((4, 4, 4, 5), (2, 2, 2, 5)), ((4, 4, 4, 6), (2, 2, 2, 2)), ((4, 4, 4, 8), (2, 2, 2, 3))):
        rc = lib.mbbs_lattice_create((ctypes.c_int * 4)(*dims), (ctypes.c_int * 4)(*block), fake, 0.1, ph, None,
                                     ctypes.byref(out))
        assert rc == binding.EINVAL
        assert binding.mbbs_last_error()
    bad = (ctypes.c_double * 8)(1, 0, 1, 0, 1, 0, -2, 0)
    rc = lib.mbbs_lattice_create((ctypes.c_int * 4)(4, 4, 4, 4), (ctypes.c_int * 4)(2, 2, 2, 2), fake, 0.1, bad,
                                 None, ctypes.byref(out))
    assert rc == binding.EINVAL and "modulus" in binding.mbbs_last_error()


def test_operator_rejects_bad_block_width_before_device_work():
    """L outside 1..256 is rejected from the arguments alone (the handle and
    the pointers are not dereferenced), so this runs without a GPU."""
    import ctypes
    lib = binding.lib()
    fake = ctypes.c_void_p(16)
    for L in (0, 257):
        rc = lib.mbbs_apply_dirac(fake, L, ctypes.c_void_p(32), ctypes.c_void_p(64), binding.FP64, None)
        assert rc == binding.EINVAL
        assert "L must be" in binding.mbbs_last_error()
