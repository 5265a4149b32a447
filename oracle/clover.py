"""O(a)-improved (clover) Wilson operator and its Jacobi preconditioning (Sec. 2.2).

TEST INFRASTRUCTURE ONLY (see the package header).

The paper uses O(a)-improved Wilson fermions and divides the matrix by
(I + clover term) before the domain decomposition; it does not spell the
clover term out.  Reading taken here (the Sheikholeslami-Wohlert term in the
hopping-parameter normalisation of Sec. 2.1, A = 1 - kappa H):

    Q_{mu nu}(x) = sum of the four plaquettes in the (mu, nu) plane that start
                   and end at x, each traversed mu first, then nu,
    F_{mu nu}(x) = (Q_{mu nu}(x) - Q_{mu nu}(x)^dagger) / 8,
    sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu],
    T(x)          = i * c_sw * kappa * sum_{mu < nu} sigma_{mu nu} (x) F_{mu nu}(x),

    D = (1 + T) - kappa H ,    A = (1 + T)^{-1} D = 1 - kappa (1 + T)^{-1} H .

T(x) acts on spin (sigma) and colour (F) of site x only; it is hermitian and
commutes with gamma_5.  Plaquettes use the links as given (the fermion
boundary phases are not part of the gauge field).  The Jacobi-preconditioned
system is A X = (1 + T)^{-1} B.

Site matrices are (V, 12, 12) with row index 3*spin + colour.
"""

from __future__ import annotations

import numpy as np

from . import dirac
from . import gamma as _gamma
from . import geometry


def _shift(U, dims, mu, step):
    """Field at x + step*mu (periodic), for arrays indexed by site first."""
    nb = geometry.neighbours(dims)[:, 2 * mu + (0 if step > 0 else 1)]
    return U[nb]


def _dag(M):
    return np.conj(np.swapaxes(M, -1, -2))


def clover_leaf(U, dims, mu, nu):
    """Q_{mu nu}(x) for every site: (V, 3, 3)."""
    Um, Un = U[:, mu], U[:, nu]
    Un_xpm = _shift(Un, dims, mu, +1)                      # U_nu(x+mu)
    Um_xpn = _shift(Um, dims, nu, +1)                      # U_mu(x+nu)
    Um_xmm = _shift(Um, dims, mu, -1)                      # U_mu(x-mu)
    Un_xmm = _shift(Un, dims, mu, -1)                      # U_nu(x-mu)
    Um_xmm_pn = _shift(Um_xmm, dims, nu, +1)               # U_mu(x-mu+nu)
    Um_xmm_mn = _shift(Um_xmm, dims, nu, -1)               # U_mu(x-mu-nu)
    Un_xmm_mn = _shift(Un_xmm, dims, nu, -1)               # U_nu(x-mu-nu)
    Un_xmn = _shift(Un, dims, nu, -1)                      # U_nu(x-nu)
    Um_xmn = _shift(Um, dims, nu, -1)                      # U_mu(x-nu)
    Un_xpm_mn = _shift(Un_xpm, dims, nu, -1)               # U_nu(x+mu-nu)
    p1 = Um @ Un_xpm @ _dag(Um_xpn) @ _dag(Un)
    p2 = Un @ _dag(Um_xmm_pn) @ _dag(Un_xmm) @ Um_xmm
    p3 = _dag(Um_xmm) @ _dag(Un_xmm_mn) @ Um_xmm_mn @ Un_xmn
    p4 = _dag(Un_xmn) @ Um_xmn @ Un_xpm_mn @ _dag(Um)
    return p1 + p2 + p3 + p4


def field_strength(U, dims, mu, nu):
    Q = clover_leaf(U, dims, mu, nu)
    return (Q - _dag(Q)) / 8.0


def sigma(mu, nu):
    g = _gamma.gammas()
    return 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])


def clover_term(U, dims, csw: float, kappa: float):
    """T(x) as (V, 12, 12) site matrices."""
    V = int(np.prod(dims))
    T = np.zeros((V, 12, 12), dtype=np.complex128)
    for mu in range(4):
        for nu in range(mu + 1, 4):
            F = field_strength(U, dims, mu, nu)
            T += 1j * csw * kappa * np.einsum("st,xab->xsatb", sigma(mu, nu), F).reshape(V, 12, 12)
    return T


def jacobi_inverse(U, dims, csw: float, kappa: float):
    """(1 + T(x))^{-1} per site, by a dense inverse of each 12 x 12 matrix."""
    T = clover_term(U, dims, csw, kappa)
    return np.linalg.inv(np.eye(12)[None] + T)


def jacobi_inverse_sites(U, dims, csw: float, kappa: float, sites):
    """(1 + T(x))^{-1} at the listed sites only, (n, 12, 12): the same leaves,
    field strength and sigma sum as `jacobi_inverse`, with the neighbours of
    each listed site looked up in the periodic neighbour table, so that large
    lattices can be checked at a sample of sites."""
    sites = np.asarray(sites, dtype=np.int64)
    nb = geometry.neighbours(dims)
    fwd = lambda x, mu: nb[x, 2 * mu]          # noqa: E731
    bwd = lambda x, mu: nb[x, 2 * mu + 1]      # noqa: E731
    n = len(sites)
    T = np.zeros((n, 12, 12), dtype=np.complex128)
    x = sites
    for mu in range(4):
        for nu in range(mu + 1, 4):
            xm, xn = bwd(x, mu), bwd(x, nu)
            p1 = U[x, mu] @ U[fwd(x, mu), nu] @ _dag(U[fwd(x, nu), mu]) @ _dag(U[x, nu])
            p2 = U[x, nu] @ _dag(U[fwd(xm, nu), mu]) @ _dag(U[xm, nu]) @ U[xm, mu]
            p3 = _dag(U[xm, mu]) @ _dag(U[bwd(xm, nu), nu]) @ U[bwd(xm, nu), mu] @ U[xn, nu]
            p4 = _dag(U[xn, nu]) @ U[xn, mu] @ U[fwd(xn, mu), nu] @ _dag(U[x, mu])
            Q = p1 + p2 + p3 + p4
            F = (Q - _dag(Q)) / 8.0
            T += 1j * csw * kappa * np.einsum("st,xab->xsatb", sigma(mu, nu), F).reshape(n, 12, 12)
    return np.linalg.inv(np.eye(12)[None] + T)


def site_mul(M, phi):
    """(M phi)(x) = M(x) phi(x) for (V, 12, 12) M and (V, 4, 3, L) phi."""
    V = M.shape[0]
    L = phi.shape[-1]
    return (M @ phi.reshape(V, 12, L)).reshape(V, 4, 3, L)


def apply_D(U, kappa, phases, T, phi, dims):
    """D phi = (1 + T) phi - kappa H phi (unpreconditioned clover operator)."""
    V = int(np.prod(dims))
    phi = dirac.as_field(phi, V)
    return phi + site_mul(T, phi) - kappa * dirac.hopping(U, phases, phi, dims)


def apply_A(U, kappa, phases, cinv, phi, dims):
    """A phi = phi - kappa (1 + T)^{-1} H phi (Jacobi preconditioned)."""
    V = int(np.prod(dims))
    phi = dirac.as_field(phi, V)
    return phi - kappa * site_mul(cinv, dirac.hopping(U, phases, phi, dims))
