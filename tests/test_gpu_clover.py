"""GPU clover term and Jacobi-preconditioned operator (Sec. 2.2) against the
oracle: the site inverses (1 + T)^{-1} built on the device from the links,
the operator A = 1 - kappa (1 + T)^{-1} H in every storage precision, its
Dirichlet blocks, SAP with MR and SSOR domain solves, and a full solve."""

import numpy as np
import pytest

from oracle import clover, dirac, krylov, sap, ssor
from paper_1104_0737_amd import configs, inputs

pytestmark = pytest.mark.gpu
gu = pytest.importorskip("tests.gpu_util")
torch = gu.torch
B = gu.binding

PH_TWIST = ((np.cos(0.3), np.sin(0.3)), (1.0, 0.0), (np.cos(1.1), -np.sin(1.1)), (-1.0, 0.0))
TOL = {B.FP64: 1e-13, B.FP32: 1e-6, B.FP16S: 2e-3}
CSW = 1.3


@pytest.mark.parametrize("dims,block", [((4, 4, 4, 4), (2, 2, 2, 2)), ((8, 8, 4, 4), (4, 4, 2, 2)),
                                        ((4, 6, 4, 8), (2, 3, 2, 4))])
def test_clover_inverse_parity(dims, block):
    gu.flush(f"clover inverse {dims}")
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, 0.4, 61)
    ref = clover.jacobi_inverse(U, dims, CSW, 0.12)
    with gu.Lattice(dims, block, U, 0.12) as lat:
        B.mbbs_lattice_set_clover(lat.h, CSW)
        out = torch.empty((V, 12, 12), dtype=torch.complex128, device="cuda")
        B.mbbs_lattice_clover_inverse(lat.h, out)
        got = gu.host(out)
    np.testing.assert_allclose(got, ref, atol=1e-13)


@pytest.mark.parametrize("dims,block,L", [((8, 8, 4, 4), (4, 4, 2, 2), 4), ((4, 6, 4, 8), (2, 3, 2, 4), 5),
                                          ((8, 8, 8, 8), (4, 4, 4, 4), 12)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_clover_operator_parity(dims, block, L, prec):
    gu.flush(f"clover operator {dims} L={L} prec={prec}")
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, 0.35, 62)
    cinv = clover.jacobi_inverse(U, dims, CSW, 0.1235)
    X = inputs.gaussian_block(V, L, 63)
    ref = clover.apply_A(U, 0.1235, PH_TWIST, cinv, X, dims).reshape(12 * V, L)
    dom = sap.Domains(dims, block)
    refb = sap.apply_blocked(U, 0.1235, PH_TWIST, dom, X, cinv).reshape(12 * V, L)
    with gu.Lattice(dims, block, U, 0.1235, PH_TWIST) as lat:
        B.mbbs_lattice_set_clover(lat.h, CSW)
        B.mbbs_lattice_tune(lat.h, B.TUNE_SPLIT[prec], 2)   # must fall back to the clover-capable kernels
        Xd = gu.dev(X)
        Yd = torch.empty_like(Xd)
        B.mbbs_apply_dirac(lat.h, L, Xd, Yd, prec)
        assert np.all(gu.rel_col_err(gu.host(Yd), ref) <= TOL[prec])
        B.mbbs_apply_blocked(lat.h, L, Xd, Yd, prec)
        assert np.all(gu.rel_col_err(gu.host(Yd), refb) <= TOL[prec])
        B.mbbs_apply_clover_inverse(lat.h, L, Xd, Yd)
        np.testing.assert_allclose(gu.host(Yd), clover.site_mul(cinv, X.reshape(V, 4, 3, L)).reshape(12 * V, L),
                                   atol=1e-13)


def test_clover_removed_gives_wilson_bitwise():
    dims, block, L = (8, 8, 4, 4), (4, 4, 2, 2), 3
    V = int(np.prod(dims))
    U = inputs.gauge_field(dims, 0.35, 64)
    X = gu.dev(inputs.gaussian_block(V, L, 65))
    with gu.Lattice(dims, block, U, 0.12) as lat:
        Y0 = torch.empty_like(X)
        B.mbbs_apply_dirac(lat.h, L, X, Y0, 0)
        B.mbbs_lattice_set_clover(lat.h, CSW)
        Y1 = torch.empty_like(X)
        B.mbbs_apply_dirac(lat.h, L, X, Y1, 0)
        B.mbbs_lattice_set_clover(lat.h, 0.0)
        Y2 = torch.empty_like(X)
        B.mbbs_apply_dirac(lat.h, L, X, Y2, 0)
        a, b, c = gu.host(Y0), gu.host(Y1), gu.host(Y2)
    assert a.tobytes() == c.tobytes()
    assert np.abs(a - b).max() > 1e-3


@pytest.mark.parametrize("solver", ["mr_fused", "mr", "ssor"])
@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 3e-5), (2, 1e-2)])
def test_clover_sap_parity(solver, prec, tol):
    dims, block, L = (8, 8, 8, 8), (4, 4, 4, 4), 4
    gu.flush(f"clover sap {solver} prec={prec}")
    V = 4096
    U = inputs.gauge_field(dims, 0.3, 66)
    cinv = clover.jacobi_inverse(U, dims, CSW, 0.12)
    eta = inputs.gaussian_block(V, L, 67)
    dom = sap.Domains(dims, block)
    with gu.Lattice(dims, block, U, 0.12) as lat:
        B.mbbs_lattice_set_clover(lat.h, CSW)
        Yd = torch.empty((12 * V, L), dtype=torch.complex128, device="cuda")
        if solver == "ssor":
            solve = ssor.ssor_domain_solver(U, 0.12, gu.PH_AP, dom, 1.26, 1, cinv)
            ref = sap.sap(U, 0.12, gu.PH_AP, dom, eta, 3, 0, domain_solve=solve, cinv=cinv).reshape(12 * V, L)
            ws = torch.empty(B.mbbs_ssor_workspace_size(lat.h, L, prec), dtype=torch.uint8, device="cuda")
            B.mbbs_sap_apply_ssor(lat.h, L, gu.dev(eta), Yd, 3, 1, 1.26, prec, ws)
        else:
            B.mbbs_lattice_tune(lat.h, B.TUNE_MR_FUSED, 1 if solver == "mr_fused" else 0)
            ref = sap.sap(U, 0.12, gu.PH_AP, dom, eta, 3, 4, cinv=cinv).reshape(12 * V, L)
            ws = torch.empty(B.mbbs_sap_workspace_size(lat.h, L, prec), dtype=torch.uint8, device="cuda")
            B.mbbs_sap_apply(lat.h, L, gu.dev(eta), Yd, 3, 4, prec, ws)
        err = gu.rel_col_err(gu.host(Yd), ref)
    assert np.all(err <= tol), err


@pytest.mark.parametrize("domain_solver", [0, 1])
def test_clover_solve(domain_solver):
    """The c1 system with a clover term (c_sw = 1.3): A X = (1 + T)^{-1} B to
    1e-10 by the oracle's own residual, FP32 SAP with MR or SSOR domains."""
    cfg = configs.c1()
    U = cfg.gauge()
    Bh = cfg.sources()
    cinv = clover.jacobi_inverse(U, cfg.dims, CSW, cfg.kappa)
    Bp = clover.site_mul(cinv, Bh.reshape(cfg.V, 4, 3, cfg.L)).reshape(12 * cfg.V, cfg.L)
    with gu.Lattice(cfg.dims, cfg.block, U, cfg.kappa) as lat:
        B.mbbs_lattice_set_clover(lat.h, CSW)
        p = B.mbbs_solve_params_default(tol=1e-10, sap_prec=B.FP32, domain_solver=domain_solver)
        ws = torch.empty(B.mbbs_solve_workspace_size(lat.h, cfg.L, p), dtype=torch.uint8, device="cuda")
        Bd = gu.dev(Bh)
        Xd = torch.empty_like(Bd)
        info = B.mbbs_solve(lat.h, cfg.L, Bd, Xd, p, ws)
        X = gu.host(Xd)
    assert info["status"] == B.OK
    r = Bp - clover.apply_A(U, cfg.kappa, cfg.phases, cinv, X, cfg.dims).reshape(12 * cfg.V, cfg.L)
    tr = np.linalg.norm(r, axis=0) / np.linalg.norm(Bp, axis=0)
    gu.flush(f"  clover solve ({'SSOR' if domain_solver else 'MR'}): {info['iterations']} iterations, "
             f"true residual {tr.max():.2e}")
    assert np.all(tr <= 1.01e-10), tr
    # the unpreconditioned clover operator: D X = B to the same relative accuracy up to cond(1 + T)
    T = clover.clover_term(U, cfg.dims, CSW, cfg.kappa)
    rd = Bh - clover.apply_D(U, cfg.kappa, cfg.phases, T, X, cfg.dims).reshape(12 * cfg.V, cfg.L)
    assert np.all(np.linalg.norm(rd, axis=0) / np.linalg.norm(Bh, axis=0) <= 1e-9)


@pytest.mark.slow
def test_clover_operator_full_size_sampled():
    """32^3 x 64, L = 12, c_sw = 1.0 (the benchmark's clover option): the site
    inverses built on the device and the Jacobi-preconditioned operator in
    FP64, FP32 and FP16 storage, against the oracle at sampled sites
    (boundary sites among them)."""
    cfg = configs.c4()
    dims, L, V, csw = cfg.dims, 12, cfg.V, 1.0
    gu.flush("clover full size: links")
    U = cfg.gauge()
    rng = np.random.default_rng(4010)
    sites = np.concatenate([[0, V - 1, 31, 32 * 32 * 32 * 63], rng.integers(0, V, 150)]).astype(np.int64)
    gu.flush("clover full size: oracle site inverses")
    cinv = clover.jacobi_inverse_sites(U, dims, csw, cfg.kappa, sites)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(4011)
    with gu.Lattice(dims, cfg.block, U, cfg.kappa) as lat:
        B.mbbs_lattice_set_clover(lat.h, csw)
        gu.flush("clover full size: device inverses")
        Cd = torch.empty((V, 12, 12), dtype=torch.complex128, device="cuda")
        B.mbbs_lattice_clover_inverse(lat.h, Cd)
        got = gu.host(Cd.index_select(0, torch.from_numpy(sites).cuda()))
        np.testing.assert_allclose(got, cinv, rtol=0, atol=1e-13)
        del Cd
        Xd = torch.randn((12 * V, L), dtype=torch.complex128, device="cuda", generator=gen)
        X = gu.host(Xd)
        # A X = X + (1 + T)^{-1} (D_wilson X - X) at the sampled sites
        DX = dirac.apply_D_sites(U, cfg.kappa, cfg.phases, X.reshape(V, 4, 3, L), dims, sites).reshape(-1, 12, L)
        Xs = X.reshape(V, 12, L)[sites]
        ref = (Xs + cinv @ (DX - Xs)).reshape(-1, L)
        idx = torch.from_numpy((12 * sites[:, None] + np.arange(12)[None, :]).ravel()).cuda()
        Yd = torch.empty_like(Xd)
        for prec in (B.FP64, B.FP32, B.FP16S):
            gu.flush(f"clover full size: operator prec {prec}")
            B.mbbs_apply_dirac(lat.h, L, Xd, Yd, prec)
            err = gu.rel_col_err(gu.host(Yd.index_select(0, idx)), ref)
            assert np.all(err <= TOL[prec]), (prec, err)


@pytest.mark.slow
def test_clover_solve_full_size():
    """The benchmark's system with the clover term (c_sw = 1.0), FP32 SAP with
    MR domains: A X = (1 + T)^{-1} B solved to 1e-10.  The residual of the
    GPU solution is formed on the GPU in FP64 and compared with the oracle's
    at sampled sites (the source site and its 8 neighbours among them)."""
    cfg = configs.c4()
    dims, L, V, csw = cfg.dims, cfg.L, cfg.V, 1.0
    gu.flush("clover solve full size: links")
    U = cfg.gauge()
    Bh = cfg.sources()
    src = cfg.src_site()
    c = np.array(np.unravel_index(src, dims[::-1])[::-1])
    sites = [src]
    for mu in range(4):
        for d in (1, -1):
            n = c.copy()
            n[mu] = (n[mu] + d) % dims[mu]
            sites.append(int(np.ravel_multi_index(tuple(n[::-1]), dims[::-1])))
    sites = np.array(sites + np.random.default_rng(4012).integers(0, V, 120).tolist(), dtype=np.int64)
    cinv = clover.jacobi_inverse_sites(U, dims, csw, cfg.kappa, sites)
    with gu.Lattice(dims, cfg.block, U, cfg.kappa) as lat:
        B.mbbs_lattice_set_clover(lat.h, csw)
        gu.flush("clover solve full size: solve")
        p = B.mbbs_solve_params_default(tol=1e-10, sap_prec=B.FP32, ncy=cfg.ncy, nmr=cfg.nmr)
        ws = torch.empty(B.mbbs_solve_workspace_size(lat.h, L, p), dtype=torch.uint8, device="cuda")
        Bd = gu.dev(Bh)
        Xd = torch.empty_like(Bd)
        info = B.mbbs_solve(lat.h, L, Bd, Xd, p, ws)
        gu.flush(f"  iterations {info['iterations']} restarts {info['restarts']} {info['seconds']:.2f}s")
        assert info["status"] == B.OK and np.all(info["true_res"] <= 1e-10)
        del ws
        X = gu.host(Xd)
        # the device's FP64 residual (1 + T)^{-1} B - A X at the sampled sites
        Bp_d = torch.empty_like(Bd)
        B.mbbs_apply_clover_inverse(lat.h, L, Bd, Bp_d)
        Yd = torch.empty_like(Xd)
        B.mbbs_apply_dirac(lat.h, L, Xd, Yd, B.FP64)
        idx = torch.from_numpy((12 * sites[:, None] + np.arange(12)[None, :]).ravel()).cuda()
        Rg = gu.host((Bp_d - Yd).index_select(0, idx))
    gu.flush("clover solve full size: oracle residual at sampled sites")
    DX = dirac.apply_D_sites(U, cfg.kappa, cfg.phases, X.reshape(V, 4, 3, L), dims, sites).reshape(-1, 12, L)
    Xs = X.reshape(V, 12, L)[sites]
    AX = Xs + cinv @ (DX - Xs)
    Bp = cinv @ Bh.reshape(V, 12, L)[sites]
    Ro = (Bp - AX).reshape(-1, L)
    # ||(1 + T)^{-1} B_j|| is O(1) (a unit source at one site); FP64 rounding of A X is ~1e-15
    assert np.max(np.abs(Rg - Ro)) <= 1e-13
    bn = np.linalg.norm(cinv[0] @ Bh.reshape(V, 12, L)[src], axis=0)   # the whole of (1 + T)^{-1} B
    assert np.all(np.linalg.norm(Ro, axis=0) / bn <= 1e-10)
