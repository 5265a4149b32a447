"""MR domain solves that form psi once per domain solve (MBBS_TUNE_MR_ONCE_*).

psi = sum_k omega_k r_k is regrouped as c r_0 - sum_j e_j w_j from the kept
residual r_0 and the steps' A r; in exact arithmetic this is the step-by-step
MR of Sec. 2.2, so SAP must match the oracle at the usual bounds (FP64,
FP32, FP16 storage; untiled and tiled stencil steps; L even and odd; one to
four steps, and five steps, which fall back to the step-by-step form), a
batch handle must equal its single handles bit for bit, and a solve must
converge to the oracle's residual bound.
"""

import numpy as np
import pytest

from oracle import sap
from paper_1104_0737_amd import configs, inputs

pytestmark = pytest.mark.gpu
gu = pytest.importorskip("tests.gpu_util")
torch = gu.torch
B = gu.binding

SAP_TOL = {B.FP64: 1e-12, B.FP32: 3e-5, B.FP16S: 1e-2}


def _sap(lat, L, eta, ncy, nmr, prec, V):
    ws = torch.empty(B.mbbs_sap_workspace_size(lat.h, L, prec), dtype=torch.uint8, device="cuda")
    Y = torch.empty((12 * V, L), dtype=torch.complex128, device="cuda")
    B.mbbs_sap_apply(lat.h, L, gu.dev(eta), Y, ncy, nmr, prec, ws)
    return gu.host(Y)


def test_knob_and_workspace():
    dims, block = (8, 8, 8, 8), (4, 4, 4, 4)
    U = inputs.gauge_field(dims, 0.3, 500)
    with gu.Lattice(dims, block, U, 0.12) as lat:
        with pytest.raises(B.MbbsError) as e:
            B.mbbs_lattice_tune(lat.h, B.TUNE_MR_ONCE[1], 2)
        assert e.value.code == B.EINVAL
        small = B.mbbs_sap_workspace_size(lat.h, 12, 1)
        B.mbbs_lattice_tune(lat.h, B.TUNE_MR_ONCE[0], 1)          # another precision's setting
        assert B.mbbs_sap_workspace_size(lat.h, 12, 1) == small
        B.mbbs_lattice_tune(lat.h, B.TUNE_MR_ONCE[1], 1)
        big = B.mbbs_sap_workspace_size(lat.h, 12, 1)
        field = 4096 * 12 * 12 * 8
        assert big - small >= 4 * field
        # a workspace sized without the setting still serves (step-by-step form)
        eta = inputs.gaussian_block(4096, 12, 501)
        ws = torch.empty(small, dtype=torch.uint8, device="cuda")
        Y = torch.empty((12 * 4096, 12), dtype=torch.complex128, device="cuda")
        B.mbbs_sap_apply(lat.h, 12, gu.dev(eta), Y, 2, 3, 1, ws)
        ref = sap.sap(U, 0.12, gu.PH_AP, sap.Domains(dims, block), eta, 2, 3).reshape(12 * 4096, 12)
        assert np.all(gu.rel_col_err(gu.host(Y), ref) <= SAP_TOL[1])


CASES = [((8, 8, 8, 8), (4, 4, 4, 4), 12), ((8, 8, 4, 8), (4, 4, 2, 4), 5), ((16, 8, 8, 8), (8, 4, 4, 4), 6)]


@pytest.mark.parametrize("dims,block,L", CASES)
@pytest.mark.parametrize("nmr", [1, 2, 4, 5])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_sap_parity(dims, block, L, nmr, prec):
    gu.flush(f"mr once {dims} L={L} nmr={nmr} prec={prec}")
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, 0.3, 502)
    eta = inputs.gaussian_block(V, L, 503)
    ncy = 2
    ref = sap.sap(U, 0.12, gu.PH_AP, sap.Domains(dims, block), eta, ncy, nmr).reshape(12 * V, L)
    with gu.Lattice(dims, block, U, 0.12) as lat:
        B.mbbs_lattice_tune(lat.h, B.TUNE_MR_FUSED, 0)
        B.mbbs_lattice_tune(lat.h, B.TUNE_MR_ONCE[prec], 1)
        for tile in (0, 1, 3, 11):
            # 11: tiled with half the columns per workgroup (where L splits so)
            B.mbbs_lattice_tune(lat.h, B.TUNE_TILE[prec], tile % 10)
            B.mbbs_lattice_tune(lat.h, B.TUNE_TILE_COLS[prec], L // 2 if tile == 11 else 0)
            Y = _sap(lat, L, eta, ncy, nmr, prec, V)
            assert np.all(gu.rel_col_err(Y, ref) <= SAP_TOL[prec]), tile
            assert np.all(gu.max_elem_err(Y, ref) <= SAP_TOL[prec]), tile


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_point_sources(prec):
    """Most domains hold an exactly zero residual (omega = 0 in every step)."""
    dims, block, L = (8, 8, 8, 8), (4, 4, 4, 4), 4
    V = 4096
    U = inputs.gauge_field(dims, 0.3, 504)
    eta = inputs.point_sources(V, L, 0, 0)
    ref = sap.sap(U, 0.11, gu.PH_AP, sap.Domains(dims, block), eta, 4, 4).reshape(12 * V, L)
    with gu.Lattice(dims, block, U, 0.11) as lat:
        B.mbbs_lattice_tune(lat.h, B.TUNE_MR_FUSED, 0)
        B.mbbs_lattice_tune(lat.h, B.TUNE_MR_ONCE[prec], 1)
        Y = _sap(lat, L, eta, 4, 4, prec, V)
    assert np.all(gu.rel_col_err(Y, ref) <= SAP_TOL[prec])


@pytest.mark.parametrize("prec", [1, 2])
def test_batch_bit_identical(prec):
    dims, block, L = (8, 8, 4, 8), (4, 4, 2, 4), 12
    V = int(np.prod(dims))
    Us = [inputs.gauge_field(dims, 0.3, 510 + k) for k in range(3)]
    ks = [0.112 + 0.004 * k for k in range(3)]
    singles = [gu.Lattice(dims, block, U, kk) for U, kk in zip(Us, ks)]
    U_dev = [gu.dev(U) for U in Us]
    h = B.mbbs_lattice_create_batch(dims, block, U_dev, ks, gu.PH_AP)
    try:
        etas = [inputs.gaussian_block(V, L, 520 + k) for k in range(3)]
        for hh in [h] + [s.h for s in singles]:
            B.mbbs_lattice_tune(hh, B.TUNE_MR_FUSED, 0)
            B.mbbs_lattice_tune(hh, B.TUNE_MR_ONCE[prec], 1)
        ws = torch.empty(B.mbbs_sap_workspace_size(h, L, prec), dtype=torch.uint8, device="cuda")
        Y = torch.empty((3 * 12 * V, L), dtype=torch.complex128, device="cuda")
        B.mbbs_sap_apply(h, L, gu.dev(np.concatenate(etas)), Y, 3, 4, prec, ws)
        Y = gu.host(Y)
        N = 12 * V
        for k, (lat, eta) in enumerate(zip(singles, etas)):
            R = _sap(lat, L, eta, 3, 4, prec, V)
            assert Y[k * N:(k + 1) * N].tobytes() == R.tobytes(), k
    finally:
        for s in singles:
            s.close()
        B.mbbs_lattice_destroy(h)


@pytest.mark.parametrize("sap_prec", [1, 2])
def test_solve(sap_prec):
    """c3 (8^4, L = 4) with psi formed once: converged, and the oracle's own
    residual of the GPU solution within the tolerance."""
    from oracle import dirac
    cfg = configs.c3()
    U = cfg.gauge()
    Bh = cfg.sources()
    with gu.Lattice(cfg.dims, cfg.block, U, cfg.kappa) as lat:
        B.mbbs_lattice_tune(lat.h, B.TUNE_MR_FUSED, 0)
        B.mbbs_lattice_tune(lat.h, B.TUNE_MR_ONCE[sap_prec], 1)
        p = B.mbbs_solve_params_default(tol=1e-10, sap_prec=sap_prec, profile=1, ncy=cfg.ncy, nmr=cfg.nmr)
        ws = torch.empty(B.mbbs_solve_workspace_size(lat.h, cfg.L, p), dtype=torch.uint8, device="cuda")
        Xd = torch.empty((12 * cfg.V, cfg.L), dtype=torch.complex128, device="cuda")
        info = B.mbbs_solve(lat.h, cfg.L, gu.dev(Bh), Xd, p, ws)
    assert info["status"] == B.OK
    X = gu.host(Xd)
    R = Bh - dirac.apply_D(U, cfg.kappa, cfg.phases, X, cfg.dims).reshape(Bh.shape)
    assert np.all(np.linalg.norm(R, axis=0) / np.linalg.norm(Bh, axis=0) <= 1e-10 * 1.01)
    it, n = info["iterations"], info["kernel_launches"]
    # per domain solve: nmr stencil steps, nmr - 1 residual steps and one psi pass
    assert n["mr_dslash"] == 2 * it * 2 * cfg.ncy * cfg.nmr
    assert n["mr_update"] == 2 * it * 2 * cfg.ncy * cfg.nmr
