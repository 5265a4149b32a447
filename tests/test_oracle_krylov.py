"""Pins of the oracle's modified block BiCGSTAB (Alg. 1, Alg. 2) and MGS QR.

* MGS equals LAPACK Householder QR once diagonal phases are made positive;
* with L = 1 the block method reproduces textbook BiCGSTAB (van der Vorst)
  residual history, with and without a preconditioner;
* the Petrov-Galerkin conditions R~^H T = 0 (step 4.5) and Tr(Z^H R) = 0
  (step 4.10) hold every iteration;
* the solution equals a dense LU solve of the same system;
* the QR step keeps the true and recursive residuals together, while
  without it the true residual stalls (the paper's claim in its abstract
  and conclusions), on a system where the gap is clear;
* a false stop of the recursion (no QR) is repaired by the restart from the
  true residual;
* Alg. 2 (memory-saving) gives the same iterates as Alg. 1.
"""

import numpy as np
import pytest

from oracle import dirac, krylov, sap

import oracle_pins
from paper_1104_0737_amd import inputs

PH = ((1.0, 0.0), (1.0, 0.0), (1.0, 0.0), (-1.0, 0.0))
DIMS = (4, 4, 4, 4)
V = 256


@pytest.fixture(scope="module")
def system():
    return oracle_pins.krylov_system()


def test_mgs_matches_householder():
    rng = np.random.default_rng(1)
    P = rng.standard_normal((300, 7)) + 1j * rng.standard_normal((300, 7))
    Q, g = krylov.mgs(P)
    np.testing.assert_allclose(Q @ g, P, atol=1e-13)
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(7), atol=1e-14)
    assert np.allclose(np.tril(g, -1), 0) and np.all(np.diag(g).real > 0)
    Qh, Rh = np.linalg.qr(P)
    ph = np.diag(Rh) / np.abs(np.diag(Rh))
    np.testing.assert_allclose(Q, Qh * ph[None, :], atol=1e-13)
    np.testing.assert_allclose(g, Rh / ph[:, None], atol=1e-13)


@pytest.mark.parametrize("precond", ["none", "sap"])
def test_L1_reduces_to_textbook_bicgstab(system, precond):
    U, D = system
    kappa = 0.15
    A = lambda X: D @ X
    if precond == "none":
        M = lambda X: X
    else:
        dom = sap.Domains(DIMS, (2, 2, 2, 2))
        M = lambda X: sap.sap(U, kappa, PH, dom, X, 2, 3).reshape(12 * V, -1)
    b = inputs.gaussian_block(V, 1, 3)
    res = krylov.block_bicgstab(A, M, b, 1e-12, maxiter=20, max_restarts=0)
    _, hist = krylov.bicgstab(A, M, b, 1e-12, maxiter=20)
    n = min(len(hist), len(res.history), 20)
    assert n >= 8
    np.testing.assert_allclose(res.history[:n], hist[:n], rtol=1e-10)


def test_block_invariants():
    oracle_pins.check_block_invariants(krylov)


def test_solution_matches_dense_lu(system):
    U, D = system
    B = inputs.point_sources(V, 12, 17, 0)
    Xd = np.linalg.solve(D, B)
    dom = sap.Domains(DIMS, (2, 2, 2, 2))
    M = lambda X: sap.sap(U, 0.15, PH, dom, X, 4, 4).reshape(12 * V, -1)
    r = krylov.block_bicgstab(lambda X: D @ X, M, B, 1e-12, maxiter=200)
    assert r.converged and np.max(r.true_res) <= 1e-12
    cond = np.linalg.cond(D)
    err = np.linalg.norm(r.X - Xd, axis=0) / np.linalg.norm(Xd, axis=0)
    assert np.max(err) <= cond * 1e-12
    # recursive and true residual agree (QR keeps them together)
    assert np.max(np.abs(np.log10(r.true_res) - np.log10(r.rec_res))) < 1.0


def test_qr_suppresses_true_recursive_gap(system):
    _, D = system
    A = lambda X: D @ X
    B = inputs.point_sources(V, 12, 5, 0)
    with_qr = krylov.block_bicgstab(A, lambda X: X, B, 1e-14, maxiter=400, qr=True,
                                    track_true=True, max_restarts=0)
    no_qr = krylov.block_bicgstab(A, lambda X: X, B, 1e-14, maxiter=400, qr=False,
                                  track_true=True, max_restarts=0)

    def gap(r):
        return max(abs(np.log10(t) - np.log10(h)) for t, h in zip(r.true_history, r.history))
    assert gap(with_qr) < 0.5
    assert gap(no_qr) > 1.0
    assert np.max(with_qr.true_res) < 0.1 * np.max(no_qr.true_res)


def test_memsave_equals_alg1(system):
    U, D = system
    A = lambda X: D @ X
    dom = sap.Domains(DIMS, (2, 2, 2, 2))
    M = lambda X: sap.sap(U, 0.15, PH, dom, X, 2, 2).reshape(12 * V, -1)
    B = inputs.point_sources(V, 4, 40, 2)
    r1 = krylov.block_bicgstab(A, M, B, 1e-10, maxiter=50)
    r2 = krylov.block_bicgstab_memsave(A, M, B, 1e-10, maxiter=50)
    assert r1.iterations == r2.iterations
    np.testing.assert_allclose(r2.history, r1.history, rtol=1e-6)
    np.testing.assert_allclose(r2.X, r1.X, atol=1e-9 * np.max(np.abs(r1.X)))


def test_restart_and_initial_guess(system):
    _, D = system
    A = lambda X: D @ X
    B = inputs.point_sources(V, 3, 2, 0)
    r = krylov.block_bicgstab(A, lambda X: X, B, 1e-6, maxiter=200)
    # resuming from the returned X needs (almost) no further work
    r2 = krylov.block_bicgstab(A, lambda X: X, B, 1e-6, maxiter=200, X0=r.X)
    assert r2.iterations == 0 and r2.converged
    # maxiter exhausted: not converged, residuals reported
    r3 = krylov.block_bicgstab(A, lambda X: X, B, 1e-12, maxiter=2)
    assert not r3.converged and r3.iterations == 2 and np.all(r3.true_res > 1e-12)


def test_restart_from_true_residual():
    oracle_pins.check_restart(krylov)
