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


def _header_enums():
    """Every enumerator of include/mbbs.h with its value (implicit values
    counted on from the previous one)."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    vals = {}
    for body in re.findall(r"enum\s*\{(.*?)\}", text, flags=re.S):
        nxt = 0
        for item in body.split(","):
            item = item.strip()
            if not item:
                continue
            m = re.fullmatch(r"(MBBS_\w+)\s*(?:=\s*(-?\d+))?", item)
            assert m, item
            v = int(m.group(2)) if m.group(2) is not None else nxt
            vals[m.group(1)] = v
            nxt = v + 1
    return vals


def test_binding_constants_match_header_enums():
    """The binding's precisions, status codes, table ids, kernel classes and
    tuning knob numbers are the header's."""
    e = _header_enums()
    assert (e["MBBS_FP64"], e["MBBS_FP32"], e["MBBS_FP16S"]) == (binding.FP64, binding.FP32, binding.FP16S)
    for name in ("OK", "NOT_CONVERGED", "EINVAL", "ENOMEM", "EHIP", "EBREAKDOWN"):
        assert e["MBBS_" + name] == getattr(binding, name), name
    for i, t in enumerate(binding.TABLES):
        assert e["MBBS_TAB_" + t] == i, t
    assert e["MBBS_TAB_COUNT"] == len(binding.TABLES)
    header_name = {"sap_resid": "SAP_RES"}
    for i, k in enumerate(binding.KERNEL_CLASSES):
        assert e["MBBS_K_" + header_name.get(k, k.upper())] == i, k
    assert e["MBBS_K_COUNT"] == len(binding.KERNEL_CLASSES)
    per_prec = {"GROUP": binding.TUNE_GROUP, "SPLIT": binding.TUNE_SPLIT, "HOP_PAIR": binding.TUNE_HOP_PAIR,
                "NT_STORE": binding.TUNE_NT_STORE, "CHUNK": binding.TUNE_CHUNK,
                "BLOCK_THREADS": binding.TUNE_BLOCK_THREADS_PREC, "TILE": binding.TUNE_TILE,
                "MR_ONCE": binding.TUNE_MR_ONCE, "TILE_COLS": binding.TUNE_TILE_COLS}
    for knob, m in per_prec.items():
        for prec, suffix in ((binding.FP64, "FP64"), (binding.FP32, "FP32"), (binding.FP16S, "FP16S")):
            assert e[f"MBBS_TUNE_{knob}_{suffix}"] == m[prec], (knob, suffix)
    single = ("BLOCK_THREADS", "LDS_PAD_KB", "PERSIST_BLOCKS", "MR_FUSED")
    for knob in single:
        assert e["MBBS_TUNE_" + knob] == getattr(binding, "TUNE_" + knob), knob
    tune = {k for k in e if k.startswith("MBBS_TUNE_")}
    assert len(tune) == len(single) + 3 * len(per_prec)      # every knob of the header is mapped above


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """With the HIP library absent the binding raises at once: there is no
    other path (no CPU fallback) behind any entry point."""
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "libmbbs.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        binding.lib()
    with pytest.raises(RuntimeError, match="missing"):
        binding.mbbs_solve_params_default()


def test_struct_layouts_match_header(tmp_path):
    """The binding's ctypes images of mbbs_solve_params and mbbs_solve_info
    have the header's size and field offsets (checked by compiling a small
    host program against include/mbbs.h)."""
    import subprocess
    structs = {"mbbs_solve_params": binding.SolveParams, "mbbs_solve_info": binding.SolveInfo}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {(a, b): int(c) for a, b, c in (ln.split() for ln in out if ln)}
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
