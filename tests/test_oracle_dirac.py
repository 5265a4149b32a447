"""Pins of the oracle's Wilson-Dirac operator (Sec. 2.1, hopping-term equation).

* free field: plane waves are eigenvectors with a closed-form eigenvalue,
  and the spectrum of the dense matrix is the closed-form set;
* gamma5-hermiticity: gamma5 A gamma5 = A^H;
* gauge covariance under random SU(3) transformations;
* three independent codings (array rolls, per-site loop, dense matrix built
  hop by hop) agree;
* the domain-restricted operator equals sum_D P_D A P_D.
"""

import numpy as np
import pytest

from oracle import dirac, gamma, geometry
from paper_1104_0737_amd import inputs

PH_AP = ((1.0, 0.0), (1.0, 0.0), (1.0, 0.0), (-1.0, 0.0))
PH_TWIST = ((np.cos(0.3), np.sin(0.3)), (1.0, 0.0), (np.cos(1.1), -np.sin(1.1)), (-1.0, 0.0))


def _rand_block(V, L, seed):
    return inputs.gaussian_block(V, L, seed).reshape(V, 4, 3, L)


def _unit_links(V):
    return np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3)).copy()


@pytest.mark.parametrize("phases", [PH_AP, PH_TWIST])
def test_free_field_plane_wave(phases):
    dims = (4, 4, 6, 8)
    V = geometry.volume(dims)
    kappa = 0.13
    U = _unit_links(V)
    c = geometry.coords(dims)
    g = gamma.gammas()
    rng = np.random.default_rng(0)
    theta = [np.angle(complex(*p)) for p in phases]
    for _ in range(4):
        n = [rng.integers(dims[m]) for m in range(4)]
        p = np.array([(2 * np.pi * n[m] + theta[m]) / dims[m] for m in range(4)])
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        wave = np.exp(1j * (c @ p))
        phi = wave[:, None, None, None] * u[None, :, :, None]
        out = dirac.apply_D(U, kappa, phases, phi, dims)
        Ms = (1 - 2 * kappa * np.sum(np.cos(p))) * np.eye(4) \
            + 2j * kappa * sum(g[m] * np.sin(p[m]) for m in range(4))
        expect = wave[:, None, None, None] * (Ms @ u)[None, :, :, None]
        np.testing.assert_allclose(out, expect, atol=1e-14)


def test_free_field_spectrum_dense():
    dims = (2, 2, 2, 4)
    V = geometry.volume(dims)
    kappa = 0.11
    D = dirac.dense_D(_unit_links(V), kappa, PH_AP, dims)
    ev = np.linalg.eigvals(D)
    expect = []
    for n in np.ndindex(*dims):
        p = np.array([(2 * np.pi * n[m] + (np.pi if m == 3 else 0.0)) / dims[m] for m in range(4)])
        a = 1 - 2 * kappa * np.sum(np.cos(p))
        b = 2 * kappa * np.linalg.norm(np.sin(p))
        expect += [a + 1j * b] * 6 + [a - 1j * b] * 6
    ev = np.sort_complex(np.round(ev, 10))
    expect = np.sort_complex(np.round(np.array(expect), 10))
    np.testing.assert_allclose(ev, expect, atol=1e-9)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_dense_equals_vectorised(dims):
    V = geometry.volume(dims)
    U = inputs.gauge_field(dims, 0.4, 3)
    D = dirac.dense_D(U, 0.12, PH_TWIST, dims)
    phi = _rand_block(V, 3, 1)
    out = dirac.apply_D(U, 0.12, PH_TWIST, phi, dims).reshape(12 * V, 3)
    np.testing.assert_allclose(out, D @ phi.reshape(12 * V, 3), atol=1e-14)


def test_persite_equals_vectorised():
    dims = (4, 4, 4, 6)
    V = geometry.volume(dims)
    U = inputs.gauge_field(dims, 0.3, 4)
    phi = _rand_block(V, 5, 2)
    full = dirac.apply_D(U, 0.124, PH_TWIST, phi, dims)
    sites = [0, 1, 3, 17, V - 1, V // 2, 4 * 4 * 4 * 5]
    part = dirac.apply_D_sites(U, 0.124, PH_TWIST, phi, dims, sites)
    np.testing.assert_allclose(part, full[sites], atol=1e-14)


def test_gamma5_hermiticity():
    dims = (4, 4, 4, 4)
    V = geometry.volume(dims)
    U = inputs.gauge_field(dims, 0.3, 5)
    psi, phi = _rand_block(V, 2, 3), _rand_block(V, 2, 4)
    lhs = np.vdot(psi, dirac.gamma5_field(dirac.apply_D(U, 0.13, PH_TWIST, dirac.gamma5_field(phi), dims)))
    rhs = np.vdot(dirac.apply_D(U, 0.13, PH_TWIST, psi, dims), phi)
    assert abs(lhs - rhs) <= 1e-14 * abs(rhs) * 10
    # dense form on a tiny lattice
    d2 = (2, 2, 2, 4)
    U2 = inputs.gauge_field(d2, 0.3, 6)
    D = dirac.dense_D(U2, 0.13, PH_TWIST, d2)
    G5 = np.kron(np.eye(geometry.volume(d2)), np.kron(gamma.gamma5(), np.eye(3)))
    np.testing.assert_allclose(G5 @ D @ G5, D.conj().T, atol=1e-15)


def _gauge_transform(U, G, dims):
    nb = geometry.neighbours(dims)
    Up = np.empty_like(U)
    for mu in range(4):
        Up[:, mu] = G @ U[:, mu] @ np.conj(np.swapaxes(G[nb[:, 2 * mu]], 1, 2))
    return Up


def test_gauge_covariance():
    dims = (4, 4, 2, 4)
    V = geometry.volume(dims)
    U = inputs.gauge_field(dims, 0.5, 7)
    G = inputs.random_su3(V, 8)
    Up = _gauge_transform(U, G, dims)
    phi = _rand_block(V, 3, 5)
    Gphi = np.einsum("vab,vsbl->vsal", G, phi)
    lhs = dirac.apply_D(Up, 0.12, PH_TWIST, Gphi, dims)
    rhs = np.einsum("vab,vsbl->vsal", G, dirac.apply_D(U, 0.12, PH_TWIST, phi, dims))
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_blocked_is_sum_of_projected_blocks():
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    V = geometry.volume(dims)
    U = inputs.gauge_field(dims, 0.3, 9)
    phi = _rand_block(V, 2, 6)
    did = geometry.domain_id(dims, block)
    expect = np.zeros_like(phi)
    for d in range(did.max() + 1):
        P = (did == d)[:, None, None, None]
        expect += P * dirac.apply_D(U, 0.12, PH_AP, P * phi, dims)
    got = dirac.apply_blocked(U, 0.12, PH_AP, phi, dims, block)
    np.testing.assert_allclose(got, expect, atol=1e-15)


def test_columns_independent():
    # the multi-RHS operator acts column by column with the same links
    dims = (4, 4, 4, 4)
    V = geometry.volume(dims)
    U = inputs.gauge_field(dims, 0.3, 10)
    phi = _rand_block(V, 4, 7)
    full = dirac.apply_D(U, 0.12, PH_AP, phi, dims)
    for i in range(4):
        one = dirac.apply_D(U, 0.12, PH_AP, phi[..., i:i + 1], dims)
        np.testing.assert_allclose(full[..., i:i + 1], one, atol=0)
