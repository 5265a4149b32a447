"""Pins of the SSOR domain inverse (Sec. 2.2, SSOR equations) in the oracle.

* the forward / backward split: 1 - Lf - Ub is the Dirichlet operator, and a
  point source shows Lf reaching only the sites x - mu (it reads phi_{x+mu});
* the nilpotent-series inverses against dense linear solves on matrices taken
  from the independently assembled dense operator;
* the paper's three-term A^S against the product (1 - w Lf)^{-1} A_DD (1 - w Ub)^{-1};
* w = 1, N = 0 is symmetric Gauss-Seidel on the dense domain blocks;
* B -> A_DD^{-1} geometrically as N grows; kappa = 0 gives B = 1; linearity.
"""

import numpy as np
import pytest

from oracle import dirac, geometry, sap, ssor
from paper_1104_0737_amd import inputs

DIMS, BLOCK = (4, 4, 4, 4), (2, 2, 2, 2)
PH = ((1.0, 0.0), (1.0, 0.0), (1.0, 0.0), (-1.0, 0.0))
V = 256


@pytest.fixture(scope="module")
def setup():
    U = inputs.gauge_field(DIMS, 0.3, 31)
    dom = sap.Domains(DIMS, BLOCK)
    return U, dom


def test_split_adds_up_to_dirichlet_operator(setup):
    U, dom = setup
    v = inputs.gaussian_block(V, 3, 32)
    lhs = dirac.as_field(v, V) - ssor.forward_inside(U, 0.12, PH, dom, v) - ssor.backward_inside(U, 0.12, PH, dom, v)
    np.testing.assert_allclose(lhs, dirac.apply_blocked(U, 0.12, PH, v, DIMS, BLOCK), atol=1e-13)


def test_forward_part_reads_forward_neighbours(setup):
    U, dom = setup
    y = 1 + 4 * (1 + 4 * (1 + 4 * 1))           # site (1,1,1,1): upper corner of its 2^4 domain
    v = np.zeros((V, 4, 3, 1), complex)
    v[y, 0, 0, 0] = 1
    lf = ssor.forward_inside(U, 0.1, PH, dom, v)
    ub = ssor.backward_inside(U, 0.1, PH, dom, v)
    c = geometry.coords(DIMS)
    hit_f = set(np.nonzero(np.abs(lf).sum(axis=(1, 2, 3)))[0])
    hit_b = set(np.nonzero(np.abs(ub).sum(axis=(1, 2, 3)))[0])
    expect_f = {int(geometry.site_of(DIMS, c[y] - np.eye(4, dtype=int)[mu])) for mu in range(4)}
    assert hit_f == expect_f          # x = y - mu reads phi_{x+mu} = phi_y
    assert hit_b == set()             # y + mu lies in the next domain: no in-domain backward hop


def _dense_parts(U, kappa):
    """Forward / backward in-domain blocks taken from the dense operator."""
    D = dirac.dense_D(U, kappa, PH, DIMS)
    did = geometry.domain_id(DIMS, BLOCK)
    c = geometry.coords(DIMS)
    N = 12 * V
    Lf = np.zeros((N, N), complex)
    Ub = np.zeros((N, N), complex)
    for s in range(V):
        for mu in range(4):
            for step, M in ((1, Lf), (-1, Ub)):
                x = c[s].copy()
                x[mu] += step
                if x[mu] < 0 or x[mu] >= DIMS[mu]:
                    continue
                t = int(geometry.site_of(DIMS, x))
                if did[t] != did[s]:
                    continue
                M[12 * s:12 * s + 12, 12 * t:12 * t + 12] = -D[12 * s:12 * s + 12, 12 * t:12 * t + 12]
    return Lf, Ub


@pytest.fixture(scope="module")
def dense(setup):
    U, _ = setup
    return _dense_parts(U, 0.12)


def test_inverses_against_dense_solves(setup, dense):
    U, dom = setup
    Lf, Ub = dense
    v = inputs.gaussian_block(V, 2, 33)
    K = ssor.nilpotency_order(BLOCK)
    w = 1.26
    I = np.eye(12 * V)
    got_f = ssor.inv_one_minus(lambda y: ssor.forward_inside(U, 0.12, PH, dom, y), w, dirac.as_field(v, V), K)
    got_b = ssor.inv_one_minus(lambda y: ssor.backward_inside(U, 0.12, PH, dom, y), w, dirac.as_field(v, V), K)
    np.testing.assert_allclose(got_f.reshape(-1, 2), np.linalg.solve(I - w * Lf, v), atol=1e-12)
    np.testing.assert_allclose(got_b.reshape(-1, 2), np.linalg.solve(I - w * Ub, v), atol=1e-12)
    # one term short of the nilpotency order is not exact
    short = ssor.inv_one_minus(lambda y: ssor.forward_inside(U, 0.12, PH, dom, y), w, dirac.as_field(v, V), K - 1)
    assert np.abs(short.reshape(-1, 2) - np.linalg.solve(I - w * Lf, v)).max() > 1e-8


def test_symmetric_gauss_seidel_special_case(setup, dense):
    U, dom = setup
    Lf, Ub = dense
    v = inputs.gaussian_block(V, 2, 34)
    I = np.eye(12 * V)
    ref = np.linalg.solve(I - Ub, np.linalg.solve(I - Lf, v))
    got = ssor.ssor_blocked(U, 0.12, PH, dom, v, 1.0, 0)
    np.testing.assert_allclose(got.reshape(-1, 2), ref, atol=1e-12)
    # the opposite order is a different operator
    other = np.linalg.solve(I - Lf, np.linalg.solve(I - Ub, v))
    assert np.abs(other - ref).max() > 1e-3


def test_eisenstat_form(setup):
    U, dom = setup
    K = ssor.nilpotency_order(BLOCK)
    w, kap = 1.26, 0.12
    c = dirac.as_field(inputs.gaussian_block(V, 2, 35), V)
    Fi = lambda x: ssor.inv_one_minus(lambda y: ssor.forward_inside(U, kap, PH, dom, y), w, x, K)
    Bi = lambda x: ssor.inv_one_minus(lambda y: ssor.backward_inside(U, kap, PH, dom, y), w, x, K)
    three = (Fi(c) + Bi(c) + (w - 2) * Fi(Bi(c))) / w
    product = Fi(dirac.apply_blocked(U, kap, PH, Bi(c), DIMS, BLOCK))
    np.testing.assert_allclose(three, product, atol=1e-12)


@pytest.mark.parametrize("kappa,omega", [(0.05, 1.0), (0.12, 1.26)])
def test_converges_to_domain_inverse(setup, kappa, omega):
    U, dom = setup
    v = inputs.gaussian_block(V, 2, 36)
    ex = sap.exact_domain_solver(U, kappa, PH, dom)
    f = dirac.as_field(v, V)
    ref = ex(f * dom.mask(0), 0) + ex(f * dom.mask(1), 1)
    errs = [np.linalg.norm(ssor.ssor_blocked(U, kappa, PH, dom, v, omega, n) - ref) / np.linalg.norm(ref)
            for n in (0, 1, 2, 4)]
    assert all(b < 0.2 * a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-4


def test_free_of_hops_and_linear(setup):
    U, dom = setup
    P = inputs.gaussian_block(V, 2, 37)
    Q = inputs.gaussian_block(V, 2, 38)
    np.testing.assert_allclose(ssor.ssor_blocked(U, 0.0, PH, dom, P, 1.26, 1).reshape(-1, 2), P, atol=0)
    a, b = 0.3 - 1.1j, 2.0 + 0.5j
    lhs = ssor.ssor_blocked(U, 0.12, PH, dom, a * P + b * Q, 1.26, 1)
    rhs = a * ssor.ssor_blocked(U, 0.12, PH, dom, P, 1.26, 1) + b * ssor.ssor_blocked(U, 0.12, PH, dom, Q, 1.26, 1)
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_sap_with_ssor_domains_is_linear_and_preconditions(setup):
    """M_SAP with SSOR domain solves is linear (unlike MR) and brings A M close to 1."""
    U, dom = setup
    solve = ssor.ssor_domain_solver(U, 0.12, PH, dom, 1.26, 1)
    P = inputs.gaussian_block(V, 2, 39)
    Q = inputs.gaussian_block(V, 2, 40)
    M = lambda x: sap.sap(U, 0.12, PH, dom, x, 4, 0, domain_solve=solve)
    np.testing.assert_allclose(M(P + 2j * Q), M(P) + 2j * M(Q), atol=1e-12)
    r = dirac.as_field(P, V) - dirac.apply_D(U, 0.12, PH, M(P), DIMS)
    assert np.linalg.norm(r) < 0.2 * np.linalg.norm(P)


@pytest.mark.parametrize("block", [(2, 2, 2, 2), (4, 4, 4, 4), (2, 3, 2, 4), (8, 4, 4, 4)])
def test_hyperplane_order(block):
    """Every in-domain forward hop goes from hyperplane h to h + 1, the order
    is a permutation, and the offsets count the sites of each hyperplane."""
    order, off = geometry.hyperplane_order(block)
    Vb = int(np.prod(block))
    assert sorted(order.tolist()) == list(range(Vb))
    h = np.empty(Vb, int)
    for k in range(len(off) - 1):
        h[order[off[k]:off[k + 1]]] = k
    nb = geometry.local_neighbours(block)
    for mu in range(4):
        f = nb[:, 2 * mu]
        inside = f >= 0
        assert np.all(h[f[inside]] == h[inside] + 1)
    assert off[0] == 0 and off[-1] == Vb and len(off) == sum(b - 1 for b in block) + 2
