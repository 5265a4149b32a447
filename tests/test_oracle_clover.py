"""Pins of the clover term and the Jacobi-preconditioned operator in the oracle
(Sec. 2.2: O(a)-improved Wilson fermions, division by I + clover term).

* free field: every plaquette is 1, so T = 0 and A is the Wilson operator;
* T(x) is hermitian and commutes with gamma_5 for any links;
* gauge covariance: T[U^g](x) = g(x) T[U](x) g(x)^dagger and D[U^g] g = g D[U];
* gamma_5-hermiticity of D = (1 + T) - kappa H;
* closed form: a constant abelian field in the (x, y) plane,
  U_x(x) = exp(i b y) (b = 2 pi / L_y), gives F_xy = -i sin(b) and
  T = c_sw kappa sin(b) diag(-1, 1, -1, 1) in spin, 0 in every other plane;
* A = (1 + T)^{-1} D by two routes.
"""

import numpy as np
import pytest

from oracle import clover, dirac, gamma, geometry
from paper_1104_0737_amd import inputs

PH = ((1.0, 0.0), (1.0, 0.0), (1.0, 0.0), (-1.0, 0.0))
DIMS = (4, 4, 4, 4)
V = 256


def test_free_field_has_no_clover_term():
    U = np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3)).copy()
    assert np.abs(clover.clover_term(U, DIMS, 1.7, 0.13)).max() == 0


def test_hermitian_and_chiral():
    U = inputs.gauge_field(DIMS, 0.4, 51)
    T = clover.clover_term(U, DIMS, 1.3, 0.12)
    assert np.abs(T).max() > 1e-2
    np.testing.assert_allclose(T, np.conj(np.swapaxes(T, -1, -2)), atol=1e-15)
    g5 = np.kron(gamma.gamma5(), np.eye(3))
    np.testing.assert_allclose(g5 @ T, T @ g5, atol=1e-15)
    for mu in range(4):
        for nu in range(4):
            if mu != nu:
                F = clover.field_strength(U, DIMS, mu, nu)
                np.testing.assert_allclose(F, -np.conj(np.swapaxes(F, -1, -2)), atol=1e-15)
    np.testing.assert_allclose(clover.field_strength(U, DIMS, 1, 2), -clover.field_strength(U, DIMS, 2, 1),
                               atol=1e-14)


def test_gauge_covariance():
    U = inputs.gauge_field(DIMS, 0.4, 52)
    g = inputs.random_su3(V, 53)
    nb = geometry.neighbours(DIMS)
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[:, mu] = g @ U[:, mu] @ np.conj(np.swapaxes(g[nb[:, 2 * mu]], -1, -2))
    T, Tg = clover.clover_term(U, DIMS, 1.1, 0.12), clover.clover_term(Ug, DIMS, 1.1, 0.12)
    G = np.einsum("st,xab->xsatb", np.eye(4), g).reshape(V, 12, 12)
    np.testing.assert_allclose(Tg, G @ T @ np.conj(np.swapaxes(G, -1, -2)), atol=1e-13)
    phi = inputs.gaussian_block(V, 2, 54).reshape(V, 4, 3, 2)
    lhs = clover.apply_D(Ug, 0.12, PH, Tg, clover.site_mul(G, phi), DIMS)
    rhs = clover.site_mul(G, clover.apply_D(U, 0.12, PH, T, phi, DIMS))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_gamma5_hermiticity():
    U = inputs.gauge_field(DIMS, 0.4, 55)
    T = clover.clover_term(U, DIMS, 1.4, 0.12)
    g5 = np.kron(gamma.gamma5(), np.eye(3))
    G5 = np.broadcast_to(g5, (V, 12, 12))
    chi = inputs.gaussian_block(V, 1, 56).reshape(V, 4, 3, 1)
    phi = inputs.gaussian_block(V, 1, 57).reshape(V, 4, 3, 1)
    D = lambda x: clover.apply_D(U, 0.12, PH, T, x, DIMS)
    lhs = np.vdot(chi, clover.site_mul(G5, D(clover.site_mul(G5, phi))))
    rhs = np.vdot(D(chi), phi)
    assert abs(lhs - rhs) < 1e-12 * abs(rhs)


def test_constant_abelian_field_closed_form():
    dims = (4, 8, 4, 4)
    Vl = int(np.prod(dims))
    b = 2 * np.pi / dims[1]
    y = geometry.coords(dims)[:, 1]
    U = np.broadcast_to(np.eye(3, dtype=complex), (Vl, 4, 3, 3)).copy()
    U[:, 0] = np.exp(1j * b * y)[:, None, None] * np.eye(3)
    F = clover.field_strength(U, dims, 0, 1)
    np.testing.assert_allclose(F, np.broadcast_to(-1j * np.sin(b) * np.eye(3), F.shape), atol=1e-14)
    for mu, nu in ((0, 2), (0, 3), (1, 2), (1, 3), (2, 3)):
        assert np.abs(clover.field_strength(U, dims, mu, nu)).max() < 1e-15
    csw, kap = 1.2, 0.13
    T = clover.clover_term(U, dims, csw, kap)
    expect = csw * kap * np.sin(b) * np.kron(np.diag([-1.0, 1.0, -1.0, 1.0]), np.eye(3))
    np.testing.assert_allclose(T, np.broadcast_to(expect, T.shape), atol=1e-14)


def test_jacobi_preconditioned_operator():
    U = inputs.gauge_field(DIMS, 0.4, 58)
    T = clover.clover_term(U, DIMS, 1.0, 0.12)
    cinv = clover.jacobi_inverse(U, DIMS, 1.0, 0.12)
    phi = inputs.gaussian_block(V, 3, 59)
    a1 = clover.apply_A(U, 0.12, PH, cinv, phi, DIMS)
    a2 = clover.site_mul(cinv, clover.apply_D(U, 0.12, PH, T, dirac.as_field(phi, V), DIMS))
    np.testing.assert_allclose(a1, a2, atol=1e-13)
    np.testing.assert_allclose(cinv @ (np.eye(12) + T), np.broadcast_to(np.eye(12), T.shape), atol=1e-13)


def test_inverse_at_sampled_sites_equals_all_sites():
    """The per-site form used for large lattices gives the same (1 + T)^{-1}
    as the all-sites form, on a lattice with every extent different and
    sites at every boundary among the sample."""
    dims = (4, 6, 4, 8)
    U = inputs.gauge_field(dims, 0.4, 91)
    full = clover.jacobi_inverse(U, dims, 1.3, 0.124)
    V = int(np.prod(dims))
    sites = np.concatenate([[0, V - 1, 3, 4 * 6 * 4 * 7], np.random.default_rng(92).integers(0, V, 40)])
    np.testing.assert_allclose(clover.jacobi_inverse_sites(U, dims, 1.3, 0.124, sites), full[sites],
                               rtol=0, atol=1e-14)
