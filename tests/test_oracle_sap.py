"""Pins of the oracle's SAP preconditioner and MR domain solver (Sec. 2.2).

* kappa = 0: A = 1, so MR is exact in one step and M = 1;
* MR: residual norm never increases, <w, r_new> = 0 after each step, and one
  step equals LAPACK's least-squares step size on the dense domain block;
* ncy = 1 with exact domain inverses equals the block lower-triangular K
  written out from its definition, and ncy cycles equal K sum_j (1 - A K)^j;
* with exact domain inverses and many cycles, M eta tends to A^{-1} eta;
* gauge covariance of the whole preconditioner.
"""

import numpy as np

from oracle import dirac, geometry, sap

import oracle_pins
from paper_1104_0737_amd import inputs

PH = ((1.0, 0.0), (1.0, 0.0), (1.0, 0.0), (-1.0, 0.0))


def _field(V, L, seed):
    return inputs.gaussian_block(V, L, seed).reshape(V, 4, 3, L)


def test_kappa_zero_identity():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    V = geometry.volume(dims)
    U = inputs.gauge_field(dims, 0.3, 1)
    dom = sap.Domains(dims, block)
    eta = _field(V, 3, 1)
    x = sap.mr_domains(U, 0.0, PH, dom, eta, 0, 1)
    np.testing.assert_allclose(x, eta * dom.mask(0), atol=1e-15)
    psi = sap.sap(U, 0.0, PH, dom, eta, ncy=2, nmr=3)
    np.testing.assert_allclose(psi, eta, atol=1e-15)


def test_mr_monotone_and_orthogonal():
    oracle_pins.check_mr_orthogonal_monotone(sap)


def test_mr_step_is_least_squares_minimiser():
    oracle_pins.check_mr_least_squares(sap)


def test_mr_trace_matches_plain_call():
    # recording the trace does not change the result
    U, _ = oracle_pins.mr_system()
    dom = sap.Domains(oracle_pins.MR_DIMS, oracle_pins.MR_BLOCK)
    rho = _field(geometry.volume(oracle_pins.MR_DIMS), 2, 24)
    tr = []
    a = sap.mr_domains(U, 0.12, PH, dom, rho, 1, 3, trace=tr)
    b = sap.mr_domains(U, 0.12, PH, dom, rho, 1, 3)
    assert len(tr) == 3 and np.array_equal(a, b)
    # the increment lives on the colour-1 domains only
    assert np.all(a * dom.mask(0) == 0)


def test_mr_zero_domain_stays_zero():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    V = geometry.volume(dims)
    U = inputs.gauge_field(dims, 0.3, 3)
    dom = sap.Domains(dims, block)
    rho = np.zeros((V, 4, 3, 1), complex)
    rho[0, 0, 0, 0] = 1.0                     # a point source in one domain
    x = sap.mr_domains(U, 0.12, PH, dom, rho, 0, 4)
    assert np.all(np.isfinite(x))
    assert np.count_nonzero(x[dom.did != dom.did[0]]) == 0


def _dense_blocks(U, kappa, dims, block):
    D = dirac.dense_D(U, kappa, PH, dims)
    col = geometry.domain_colour(dims, block)
    rows_c = [np.nonzero(np.repeat(col, 12) == c)[0] for c in (0, 1)]
    return D, rows_c


def test_one_cycle_exact_is_K():
    dims, block = (4, 4, 2, 4), (2, 2, 1, 2)
    V = geometry.volume(dims)
    kappa = 0.12
    U = inputs.gauge_field(dims, 0.3, 4)
    dom = sap.Domains(dims, block)
    solver = sap.exact_domain_solver(U, kappa, PH, dom)
    D, (E, O) = _dense_blocks(U, kappa, dims, block)
    AEE, AOE, AOO = D[np.ix_(E, E)], D[np.ix_(O, E)], D[np.ix_(O, O)]
    BEE, BOO = np.linalg.inv(AEE), np.linalg.inv(AOO)   # block diagonal over domains
    N = 12 * V
    K = np.zeros((N, N), complex)
    K[np.ix_(E, E)] = BEE
    K[np.ix_(O, E)] = -BOO @ AOE @ BEE
    K[np.ix_(O, O)] = BOO
    eta = _field(V, 2, 5)
    got = sap.sap(U, kappa, PH, dom, eta, ncy=1, nmr=0, domain_solve=solver)
    np.testing.assert_allclose(got.reshape(N, 2), K @ eta.reshape(N, 2), atol=1e-12)
    # three cycles: K (1 + (1 - A K) + (1 - A K)^2)
    I = np.eye(N)
    M3 = K @ (I + (I - D @ K) + (I - D @ K) @ (I - D @ K))
    got3 = sap.sap(U, kappa, PH, dom, eta, ncy=3, nmr=0, domain_solve=solver)
    np.testing.assert_allclose(got3.reshape(N, 2), M3 @ eta.reshape(N, 2), atol=1e-11)


def test_many_cycles_exact_converge_to_inverse():
    dims, block = (4, 4, 2, 4), (2, 2, 1, 2)
    V = geometry.volume(dims)
    kappa = 0.1
    U = inputs.gauge_field(dims, 0.3, 6)
    dom = sap.Domains(dims, block)
    solver = sap.exact_domain_solver(U, kappa, PH, dom)
    D = dirac.dense_D(U, kappa, PH, dims)
    eta = _field(V, 1, 7)
    x = np.linalg.solve(D, eta.reshape(-1, 1))
    got = sap.sap(U, kappa, PH, dom, eta, ncy=40, nmr=0, domain_solve=solver)
    err = np.linalg.norm(got.reshape(-1, 1) - x) / np.linalg.norm(x)
    assert err < 1e-12


def test_sap_gauge_covariant():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    V = geometry.volume(dims)
    U = inputs.gauge_field(dims, 0.4, 8)
    G = inputs.random_su3(V, 9)
    nb = geometry.neighbours(dims)
    Up = np.empty_like(U)
    for mu in range(4):
        Up[:, mu] = G @ U[:, mu] @ np.conj(np.swapaxes(G[nb[:, 2 * mu]], 1, 2))
    dom = sap.Domains(dims, block)
    eta = _field(V, 2, 10)
    Geta = np.einsum("vab,vsbl->vsal", G, eta)
    lhs = sap.sap(Up, 0.12, PH, dom, Geta, 3, 4)
    rhs = np.einsum("vab,vsbl->vsal", G, sap.sap(U, 0.12, PH, dom, eta, 3, 4))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_sap_reduces_residual():
    # SAP is an approximate inverse: ||eta - A M eta|| < ||eta|| and falls with ncy
    dims, block = (8, 8, 4, 4), (4, 4, 2, 2)
    V = geometry.volume(dims)
    U = inputs.gauge_field(dims, 0.3, 11)
    dom = sap.Domains(dims, block)
    eta = _field(V, 1, 12)
    res = []
    for ncy in (1, 2, 4):
        psi = sap.sap(U, 0.11, PH, dom, eta, ncy, 4)
        res.append(np.linalg.norm(eta - dirac.apply_D(U, 0.11, PH, psi, dims)) / np.linalg.norm(eta))
    assert res[0] < 1 and res[1] < res[0] and res[2] < res[1]
