"""The roofline numerator: bench.algorithmic_bytes at the benchmark's size
(32^3 x 64, L = 12, 8^4 domains, 4 cycles of 4 MR steps) equals the bytes
obtained by counting, launch by launch, the fields, site inverses and links
each kernel must move (one read or write of each per site)."""

import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

DIMS, BLOCK, L, NCY, NMR = (32, 32, 32, 64), (8, 8, 8, 8), 12, 4, 4
V = 32 * 32 * 32 * 64
VH = V // 2
F = 1 - 6 ** 4 / 8 ** 4          # sites of an 8^4 domain with a neighbour in another domain
PS = 12 * L * 8                  # psi: FP32 complex per site


def _store(prec):
    """(spinor bytes per site, link bytes) of the SAP storage."""
    return (12 * L * 8, 72) if prec == "fp32" else (12 * L * 4 + 4 * L, 36)


def ab(cls, prec="fp32", nssor=1, clover=False):
    return bench.algorithmic_bytes(cls, L, DIMS, BLOCK, NCY, NMR, prec, nssor, clover)


def test_outer_operator():
    # FP64: read X and write Y (12 L complex of 16 B each), 4 links of 9 complex
    assert ab("dslash64") == V * (2 * 12 * L * 16 + 4 * 9 * 16)
    assert ab("dslash64", clover=True) == V * (2 * 12 * L * 16 + 4 * 9 * 16 + 72 * 8)


@pytest.mark.parametrize("prec", ["fp32", "fp16s"])
def test_mr_domain_operator(prec):
    sp, lk = _store(prec)
    assert ab("mr_dslash", prec) == VH * (sp + sp + 4 * lk)          # read r, write w, links
    assert ab("mr_dslash", prec, clover=True) == VH * (2 * sp + 4 * lk + 72 * 4)


@pytest.mark.parametrize("prec", ["fp32", "fp16s"])
def test_mr_update(prec):
    sp, _ = _store(prec)
    first = 3 * sp + PS            # read r, w; write r, psi (psi assigned)
    middle = 3 * sp + 2 * PS       # read r, w, psi; write r, psi
    last = sp + 2 * PS             # read r, psi; write psi (r no longer needed)
    per_colour = (first + 2 * middle + last) + (NCY - 1) * (3 * middle + last)
    assert ab("mr_update", prec) == pytest.approx(VH * per_colour / (NCY * NMR), rel=1e-12)


@pytest.mark.parametrize("prec", ["fp32", "fp16s"])
@pytest.mark.parametrize("tiled", [False, True])
def test_psi_once(prec, tiled):
    """psi formed once per domain solve: the MR steps carry only r; the
    tiled stencil's last step stores no A r."""
    sp, lk = _store(prec)
    steps = [2 * sp + 4 * lk] * (NMR - 1) + [(sp if tiled else 2 * sp) + 4 * lk]
    got = bench.algorithmic_bytes("mr_dslash", L, DIMS, BLOCK, NCY, NMR, prec, once=True, tiled=tiled)
    assert got == pytest.approx(VH * sum(steps) / NMR, rel=1e-12)
    # per colour and cycle: NMR - 1 steps r' = r - omega w, then psi (+)= c r_0 - sum_j e_j w_j
    launches = []
    for cy in range(NCY):
        launches += [3 * sp] * (NMR - 1)
        launches.append(NMR * sp + (PS if cy == 0 else 2 * PS))
    got = bench.algorithmic_bytes("mr_update", L, DIMS, BLOCK, NCY, NMR, prec, once=True, tiled=tiled)
    assert got == pytest.approx(VH * sum(launches) / len(launches), rel=1e-12)
    # the SAP residual: no pass on the first colour of the first cycle
    res = [2 * sp + F * PS + 4 * lk] + [2 * sp + (1 + F) * PS + 4 * lk] * (2 * (NCY - 1))
    got = bench.algorithmic_bytes("sap_resid", L, DIMS, BLOCK, NCY, NMR, prec, once=True, tiled=tiled)
    assert got == pytest.approx(VH * sum(res) / len(res), rel=1e-12)


@pytest.mark.parametrize("prec", ["fp32", "fp16s"])
def test_sap_residual(prec):
    sp, lk = _store(prec)
    launches = [2 * sp,                                 # first cycle, colour 0: psi = 0
                2 * sp + F * PS + 4 * lk]               # first cycle, colour 1: psi of colour 0 only
    launches += [2 * sp + (1 + F) * PS + 4 * lk] * (2 * (NCY - 1))
    assert ab("sap_resid", prec) == pytest.approx(VH * sum(launches) / (2 * NCY), rel=1e-12)


@pytest.mark.parametrize("nssor,fields,sweeps", [(1, 10, 4), (0, 4, 2)])
def test_ssor(nssor, fields, sweeps):
    sp, lk = _store("fp32")
    launches = []
    for cy in range(NCY):
        for col in range(2):
            if cy == 0 and col == 0:
                resid = 0
            elif cy == 0:
                resid = F * PS + 4 * lk
            else:
                resid = (1 + F) * PS + 4 * lk
            psi = PS if cy == 0 else 2 * PS
            launches.append(fields * sp + resid + psi + sweeps * 4 * lk)
    assert ab("ssor", nssor=nssor) == pytest.approx(VH * sum(launches) / (2 * NCY), rel=1e-12)


def test_bench_refuses_several_gpus():
    """The benchmark measures one GPU: asked for more it says so and exits
    non-zero before touching any device."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode != 0
    assert "one GPU only" in r.stdout
