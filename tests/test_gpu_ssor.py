"""GPU SSOR domain inverse (Sec. 2.2, SSOR equations) and SAP / solves with it,
against the oracle.

The GPU runs the triangular solves as wavefronts over the hyperplanes of each
domain; the oracle sums the nilpotent series of each inverse.  Equal in exact
arithmetic: FP64 to rounding, FP32 and FP16 storage within their precision.
"""

import numpy as np
import pytest

from oracle import dirac, krylov, sap, ssor
from paper_1104_0737_amd import configs, inputs

pytestmark = pytest.mark.gpu
gu = pytest.importorskip("tests.gpu_util")
torch = gu.torch
B = gu.binding

TOL = {B.FP64: 1e-12, B.FP32: 2e-5, B.FP16S: 2e-2}


@pytest.mark.parametrize("dims,block,L", [((4, 4, 4, 4), (2, 2, 2, 2), 3), ((8, 8, 8, 8), (4, 4, 4, 4), 4),
                                          ((4, 6, 4, 8), (2, 3, 2, 4), 5), ((16, 8, 8, 8), (8, 4, 4, 4), 12)])
@pytest.mark.parametrize("nssor,omega", [(1, 1.26), (0, 1.0)])
@pytest.mark.parametrize("prec", [B.FP64, B.FP32, B.FP16S])
def test_ssor_blocked_parity(dims, block, L, nssor, omega, prec):
    gu.flush(f"ssor blocked {dims} L={L} nssor={nssor} prec={prec}")
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, 0.3, 41)
    X = inputs.gaussian_block(V, L, 42)
    dom = sap.Domains(dims, block)
    ref = ssor.ssor_blocked(U, 0.12, gu.PH_AP, dom, X, omega, nssor).reshape(12 * V, L)
    with gu.Lattice(dims, block, U, 0.12) as lat:
        ws = torch.empty(B.mbbs_ssor_workspace_size(lat.h, L, prec), dtype=torch.uint8, device="cuda")
        Yd = torch.empty((12 * V, L), dtype=torch.complex128, device="cuda")
        B.mbbs_apply_ssor_blocked(lat.h, L, gu.dev(X), Yd, nssor, omega, prec, ws)
        err = gu.rel_col_err(gu.host(Yd), ref)
    assert np.all(err <= TOL[prec]), err


@pytest.mark.parametrize("dims,block,L,ncy", [((8, 8, 8, 8), (4, 4, 4, 4), 4, 2), ((8, 8, 4, 4), (4, 4, 2, 2), 3, 3)])
@pytest.mark.parametrize("prec", [B.FP64, B.FP32, B.FP16S])
def test_sap_ssor_parity(dims, block, L, ncy, prec):
    gu.flush(f"sap ssor {dims} L={L} prec={prec}")
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, 0.3, 43)
    eta = inputs.gaussian_block(V, L, 44)
    dom = sap.Domains(dims, block)
    solve = ssor.ssor_domain_solver(U, 0.12, gu.PH_AP, dom, 1.26, 1)
    ref = sap.sap(U, 0.12, gu.PH_AP, dom, eta, ncy, 0, domain_solve=solve).reshape(12 * V, L)
    with gu.Lattice(dims, block, U, 0.12) as lat:
        ws = torch.empty(B.mbbs_ssor_workspace_size(lat.h, L, prec), dtype=torch.uint8, device="cuda")
        Yd = torch.empty((12 * V, L), dtype=torch.complex128, device="cuda")
        B.mbbs_sap_apply_ssor(lat.h, L, gu.dev(eta), Yd, ncy, 1, 1.26, prec, ws)
        err = gu.rel_col_err(gu.host(Yd), ref)
    assert np.all(err <= 3 * TOL[prec]), err


def test_ssor_rejects_bad_arguments():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    U = np.broadcast_to(np.eye(3, dtype=complex), (256, 4, 3, 3)).copy()
    with gu.Lattice(dims, block, U, 0.1) as lat:
        ws = torch.empty(B.mbbs_ssor_workspace_size(lat.h, 2, B.FP32), dtype=torch.uint8, device="cuda")
        X = torch.zeros((3072, 2), dtype=torch.complex128, device="cuda")
        Y = torch.empty_like(X)
        for nssor, omega in ((2, 1.0), (1, 0.0), (1, 2.0), (1, float("nan"))):
            with pytest.raises(B.MbbsError) as e:
                B.mbbs_apply_ssor_blocked(lat.h, 2, X, Y, nssor, omega, B.FP32, ws)
            assert e.value.code == B.EINVAL
        small = torch.empty(1024, dtype=torch.uint8, device="cuda")
        with pytest.raises(B.MbbsError):
            B.mbbs_apply_ssor_blocked(lat.h, 2, X, Y, 1, 1.26, B.FP32, small)


@pytest.mark.parametrize("prec", [B.FP32, B.FP16S])
def test_solve_with_ssor_domains(prec):
    """The c1 system (8^4, L = 4) with SSOR (N_SSOR = 1, omega = 1.26) in SAP:
    converges to 1e-10 by the oracle's own true residual and agrees with the
    oracle's FP64 solve with the same preconditioner."""
    cfg = configs.c1()
    U = cfg.gauge()
    Bh = cfg.sources()
    dom = sap.Domains(cfg.dims, cfg.block)
    solve = ssor.ssor_domain_solver(U, cfg.kappa, cfg.phases, dom, 1.26, 1)
    A = lambda X: dirac.apply_D(U, cfg.kappa, cfg.phases, X, cfg.dims).reshape(12 * cfg.V, -1)
    M = lambda X: sap.sap(U, cfg.kappa, cfg.phases, dom, X, cfg.ncy, 0, domain_solve=solve).reshape(12 * cfg.V, -1)
    ref = krylov.block_bicgstab(A, M, Bh, 1e-10, maxiter=100)
    with gu.Lattice(cfg.dims, cfg.block, U, cfg.kappa) as lat:
        p = B.mbbs_solve_params_default(tol=1e-10, sap_prec=prec, domain_solver=1, nssor=1, ssor_omega=1.26)
        ws = torch.empty(B.mbbs_solve_workspace_size(lat.h, cfg.L, p), dtype=torch.uint8, device="cuda")
        Bd = gu.dev(Bh)
        Xd = torch.empty_like(Bd)
        info = B.mbbs_solve(lat.h, cfg.L, Bd, Xd, p, ws)
        X = gu.host(Xd)
    assert info["status"] == B.OK
    r = Bh - A(X)
    tr = np.linalg.norm(r, axis=0) / np.linalg.norm(Bh, axis=0)
    assert np.all(tr <= 1.01e-10), tr
    err = np.linalg.norm(X - ref.X, axis=0) / np.linalg.norm(ref.X, axis=0)
    gu.flush(f"  SSOR solve: {info['iterations']} iterations (oracle {ref.iterations}), error {err.max():.2e}")
    assert np.all(err <= 1e-8)
    assert abs(info["iterations"] - ref.iterations) <= 2
