"""Batch handles: several same-shape systems fused into every launch.

A batch handle stacks its systems along t; every kernel treats them as
independent systems (t hops wrap inside each system, each has its own
kappa, links, coefficients and solver flag).  The same kernels then run the
same arithmetic in the same order as on single-system handles, so a batch
must reproduce the single handles bit for bit: the operator in every
precision, the Dirichlet operator, SAP with MR and with SSOR domains, and
whole solves (iterations, X, residuals, histories), including a system that
restarts from its true residual, a system that stops early and a rejected
one.  One system is also checked against the oracle.
"""

import numpy as np
import pytest

from oracle import dirac, krylov
from paper_1104_0737_amd import inputs

pytestmark = pytest.mark.gpu
gu = pytest.importorskip("tests.gpu_util")
torch = gu.torch
B = gu.binding

PH_TWIST = ((np.cos(0.3), np.sin(0.3)), (1.0, 0.0), (np.cos(1.1), -np.sin(1.1)), (-1.0, 0.0))


class Batch:
    """Single handles and one batch handle over the same systems."""

    def __init__(self, dims, block, Us, kappas, phases=gu.PH_AP):
        self.dims, self.block, self.Us, self.kappas, self.phases = dims, block, Us, kappas, phases
        self.V = int(np.prod(dims))
        self.singles = [gu.Lattice(dims, block, U, k, phases) for U, k in zip(Us, kappas)]
        self.U_dev = [gu.dev(U) for U in Us]
        self.h = B.mbbs_lattice_create_batch(dims, block, self.U_dev, kappas, phases)

    def close(self):
        for s in self.singles:
            s.close()
        B.mbbs_lattice_destroy(self.h)

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _systems(dims, n, seed, eps=0.3):
    return [inputs.gauge_field(dims, eps, seed + k) for k in range(n)], [0.112 + 0.004 * k for k in range(n)]


def test_batch_handle_reports_its_systems():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    Us, ks = _systems(dims, 3, 300)
    with Batch(dims, block, Us, ks) as b:
        assert B.mbbs_lattice_nsys(b.h) == 3
        assert B.mbbs_lattice_nsys(b.singles[0].h) == 1
        with pytest.raises(B.MbbsError) as e:
            B.mbbs_lattice_set_clover(b.h, 1.0)
        assert e.value.code == B.EINVAL


@pytest.mark.parametrize("L", [5, 12])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_batch_operator_bit_identical(L, prec):
    gu.flush(f"batch operator L={L} prec={prec}")
    dims, block = (8, 8, 4, 4), (4, 4, 2, 2)
    Us, ks = _systems(dims, 3, 310)
    with Batch(dims, block, Us, ks, PH_TWIST) as b:
        Xs = [inputs.gaussian_block(b.V, L, 320 + k) for k in range(3)]
        Xst = gu.dev(np.concatenate(Xs))
        Yst = torch.empty_like(Xst)
        B.mbbs_apply_dirac(b.h, L, Xst, Yst, prec)
        Ybl = torch.empty_like(Xst)
        B.mbbs_apply_blocked(b.h, L, Xst, Ybl, prec)
        Y, Yb = gu.host(Yst), gu.host(Ybl)
        N = 12 * b.V
        for k, (lat, X) in enumerate(zip(b.singles, Xs)):
            Xd = gu.dev(X)
            Y1 = torch.empty_like(Xd)
            B.mbbs_apply_dirac(lat.h, L, Xd, Y1, prec)
            assert gu.host(Y1).tobytes() == Y[k * N:(k + 1) * N].tobytes(), k
            B.mbbs_apply_blocked(lat.h, L, Xd, Y1, prec)
            assert gu.host(Y1).tobytes() == Yb[k * N:(k + 1) * N].tobytes(), k
        # and the second system against the oracle
        ref = dirac.apply_D(Us[1], ks[1], PH_TWIST, Xs[1], dims).reshape(N, L)
        tol = {0: 1e-14, 1: 1e-6, 2: 2e-3}[prec]
        assert np.all(gu.rel_col_err(Y[N:2 * N], ref) <= tol)


@pytest.mark.parametrize("solver", ["mr", "ssor"])
def test_batch_sap_bit_identical(solver):
    gu.flush(f"batch SAP {solver}")
    dims, block, L = (8, 8, 8, 8), (4, 4, 4, 4), 4
    Us, ks = _systems(dims, 3, 330)
    with Batch(dims, block, Us, ks) as b:
        Xs = [inputs.gaussian_block(b.V, L, 340 + k) for k in range(3)]
        Xst = gu.dev(np.concatenate(Xs))
        Yst = torch.empty_like(Xst)
        if solver == "mr":
            ws = torch.empty(B.mbbs_sap_workspace_size(b.h, L, B.FP32), dtype=torch.uint8, device="cuda")
            B.mbbs_sap_apply(b.h, L, Xst, Yst, 3, 4, B.FP32, ws)
        else:
            ws = torch.empty(B.mbbs_ssor_workspace_size(b.h, L, B.FP32), dtype=torch.uint8, device="cuda")
            B.mbbs_sap_apply_ssor(b.h, L, Xst, Yst, 3, 1, 1.26, B.FP32, ws)
        Y = gu.host(Yst)
        N = 12 * b.V
        for k, (lat, X) in enumerate(zip(b.singles, Xs)):
            Xd = gu.dev(X)
            Y1 = torch.empty_like(Xd)
            if solver == "mr":
                w1 = torch.empty(B.mbbs_sap_workspace_size(lat.h, L, B.FP32), dtype=torch.uint8, device="cuda")
                B.mbbs_sap_apply(lat.h, L, Xd, Y1, 3, 4, B.FP32, w1)
            else:
                w1 = torch.empty(B.mbbs_ssor_workspace_size(lat.h, L, B.FP32), dtype=torch.uint8, device="cuda")
                B.mbbs_sap_apply_ssor(lat.h, L, Xd, Y1, 3, 1, 1.26, B.FP32, w1)
            assert gu.host(Y1).tobytes() == Y[k * N:(k + 1) * N].tobytes(), k


def _solve_single(lat, L, Bh, **kw):
    p = B.mbbs_solve_params_default(**kw)
    ws = torch.empty(B.mbbs_solve_workspace_size(lat.h, L, p), dtype=torch.uint8, device="cuda")
    Bd = gu.dev(Bh)
    Xd = torch.empty_like(Bd)
    try:
        info = B.mbbs_solve(lat.h, L, Bd, Xd, p, ws)
    except B.MbbsError as e:
        return None, {"status": e.code}
    return gu.host(Xd), info


def _solve_batch(b, L, Bs, **kw):
    p = B.mbbs_solve_params_default(**kw)
    ws = torch.empty(B.mbbs_solve_workspace_size(b.h, L, p), dtype=torch.uint8, device="cuda")
    Bd = gu.dev(np.concatenate(Bs))
    Xd = torch.empty_like(Bd)
    rc, infos = B.mbbs_solve(b.h, L, Bd, Xd, p, ws)
    return rc, gu.host(Xd), infos


@pytest.mark.parametrize("graph_iters", [1, 3])
@pytest.mark.parametrize("sap_prec", [B.FP32, B.FP16S])
def test_batch_solve_bit_identical(graph_iters, sap_prec):
    gu.flush(f"batch solve graph_iters={graph_iters} sap_prec={sap_prec}")
    dims, block, L = (8, 8, 8, 8), (4, 4, 4, 4), 4
    Us, ks = _systems(dims, 4, 350)
    V = 4096
    Bs = [inputs.z2_sources(V, L, 360 + k) if k % 2 else inputs.point_sources(V, L, 37 * k, k % 3) for k in range(4)]
    kw = dict(tol=1e-10, sap_prec=sap_prec, graph_iters=graph_iters)
    with Batch(dims, block, Us, ks) as b:
        rc, X, infos = _solve_batch(b, L, Bs, **kw)
        assert rc == B.OK
        N = 12 * V
        for k, lat in enumerate(b.singles):
            X1, i1 = _solve_single(lat, L, Bs[k], **kw)
            ib = infos[k]
            assert ib["status"] == B.OK and i1["status"] == B.OK
            assert ib["iterations"] == i1["iterations"], k
            assert X[k * N:(k + 1) * N].tobytes() == X1.tobytes(), k
            assert ib["true_res"].tobytes() == i1["true_res"].tobytes()
            np.testing.assert_array_equal(ib["history"], i1["history"])
    # the oracle's own residual of one batch solution
    R = Bs[2] - dirac.apply_D(Us[2], ks[2], gu.PH_AP, X[2 * N:3 * N], dims).reshape(N, L)
    assert np.all(np.linalg.norm(R, axis=0) / np.linalg.norm(Bs[2], axis=0) <= 1e-10 * 1.01)


def test_batch_restart_early_stop_and_rejected_system():
    """Three systems without the QR step and without a preconditioner at
    tol = 1e-14: the first stalls and must restart from its true residual
    (as in the single-handle restart test), the second is the same system
    with other links, the third has a zero column and is rejected alone.
    Each equals its single-handle run bit for bit; the first also matches the
    oracle's restart."""
    gu.flush("batch restart / rejected system")
    dims, block, L, tol = (4, 4, 4, 4), (2, 2, 2, 2), 6, 1e-14
    Us = [inputs.gauge_field(dims, 0.3, 31), inputs.gauge_field(dims, 0.3, 32), inputs.gauge_field(dims, 0.3, 33)]
    ks = [0.15, 0.13, 0.13]
    Bs = [inputs.z2_sources(256, L, 9), inputs.z2_sources(256, L, 10), inputs.z2_sources(256, L, 11)]
    Bs[2][:, 3] = 0
    kw = dict(tol=tol, precond=0, qr_passes=0, max_restarts=6, maxiter=400)
    with Batch(dims, block, Us, ks) as b:
        rc, X, infos = _solve_batch(b, L, Bs, **kw)
        assert rc == B.EINVAL
        assert infos[2]["status"] == B.EINVAL
        N = 12 * 256
        for k in range(2):
            X1, i1 = _solve_single(b.singles[k], L, Bs[k], **kw)
            assert infos[k]["status"] == i1["status"] == B.OK
            assert infos[k]["restarts"] == i1["restarts"] and infos[k]["iterations"] == i1["iterations"]
            assert X[k * N:(k + 1) * N].tobytes() == X1.tobytes(), k
        assert infos[0]["restarts"] >= 1
    D = dirac.dense_D(Us[0], ks[0], gu.PH_AP, dims)
    ref = krylov.block_bicgstab(lambda Y: D @ Y, lambda Y: Y, Bs[0], tol, maxiter=400, qr=False, max_restarts=6)
    assert ref.restarts >= 1
    tr = np.linalg.norm(Bs[0] - D @ X[:N], axis=0) / np.linalg.norm(Bs[0], axis=0)
    assert np.all(tr <= tol * 1.01)


def test_batched_jobs_of_batch_handles():
    """mbbs_solve_batched over two batch handles and one single handle: the
    records come per system in argument order and equal the direct solves."""
    gu.flush("batched jobs of batch handles")
    L = 4
    specs = [((8, 8, 4, 4), (4, 4, 2, 2), 3, 400), ((4, 4, 4, 8), (2, 2, 2, 4), 2, 410), ((4, 4, 4, 4), (2, 2, 2, 2), 1, 420)]
    handles, Bst, singles_ref = [], [], []
    try:
        for dims, block, n, seed in specs:
            Us, ks = _systems(dims, n, seed)
            V = int(np.prod(dims))
            Bs = [inputs.z2_sources(V, L, seed + 50 + k) for k in range(n)]
            b = Batch(dims, block, Us, ks)
            handles.append(b)
            Bst.append(np.concatenate(Bs))
            rc, X, infos = _solve_batch(b, L, Bs, tol=1e-10) if n > 1 else (None, None, None)
            if n == 1:
                X, info = _solve_single(b.singles[0], L, Bs[0], tol=1e-10)
                infos = [info]
            singles_ref.append((X, infos))
        lats = [b.h if len(b.singles) > 1 else b.singles[0].h for b in handles]
        params = [B.mbbs_solve_params_default(tol=1e-10, graph_iters=2) for _ in lats]
        ws = torch.empty(B.mbbs_solve_batched_workspace_size(lats, [L] * 3, params), dtype=torch.uint8, device="cuda")
        Bd = [gu.dev(x) for x in Bst]
        Xd = [torch.empty_like(x) for x in Bd]
        rc, infos = B.mbbs_solve_batched(lats, [L] * 3, Bd, Xd, params, ws)
        assert rc == B.OK and len(infos) == 6
        pos = 0
        for (Xr, ir), x in zip(singles_ref, Xd):
            assert gu.host(x).tobytes() == Xr.tobytes()
            for r in ir:
                assert infos[pos]["iterations"] == r["iterations"] and infos[pos]["status"] == B.OK
                pos += 1
    finally:
        for b in handles:
            b.close()
