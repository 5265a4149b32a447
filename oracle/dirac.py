"""Wilson-Dirac operator, written from Sec. 2.1 (hopping-term equation).

(A phi)_x = phi_x - kappa * eta_x,
eta_x = sum_mu [ (1 - gamma_mu) U_{x,mu} phi_{x+mu}
               + (1 + gamma_mu) U^dagger_{x-mu,mu} phi_{x-mu} ].

The multi-RHS form (Sec. 2.1, block hopping-term equation) applies the same
links to every column i = 1..L; here the column is the last array axis.

Boundary phases: a forward hop that wraps from x_mu = L_mu - 1 to 0 is
multiplied by phase[mu]; a backward hop that wraps from x_mu = 0 is multiplied
by conj(phase[mu]).  (1,1,1,-1) gives antiperiodic time.  Colour action:
(U phi)_a = sum_b U_ab phi_b, (U^dagger phi)_a = sum_b conj(U_ba) phi_b.

Three independent forms are given: the vectorised `apply_D` (array rolls),
`apply_D_sites` (explicit per-site loop over a list of sites) and `dense_D`
(explicit matrix assembled site by site), so tests can compare them.
"""

from __future__ import annotations

import numpy as np

from . import gamma as _gamma
from . import geometry

_PM, _PP = _gamma.projectors()   # (1 - gamma_mu), (1 + gamma_mu)


def _axis(mu: int) -> int:
    # fields are viewed as (Lt, Lz, Ly, Lx, spin, colour, L): x is axis 3
    return 3 - mu


def as_field(v: np.ndarray, V: int) -> np.ndarray:
    """(N, L) or (V, 4, 3, L) -> (V, 4, 3, L) view."""
    return v.reshape(V, 4, 3, -1)


def _spin(P: np.ndarray, h: np.ndarray) -> np.ndarray:
    # (P h)_{s a l} = sum_t P_st h_{t a l}, h shape (..., 4, 3, L)
    sh = h.shape
    return (P @ h.reshape(sh[:-3] + (4, sh[-2] * sh[-1]))).reshape(sh)


def _colour(W: np.ndarray, h: np.ndarray) -> np.ndarray:
    # (W h)_{s a l} = sum_b W_ab h_{s b l}, W shape (..., 3, 3), h (..., 4, 3, L)
    return W[..., None, :, :] @ h


def hopping(U, phases, phi, dims, keep=None) -> np.ndarray:
    """eta = H phi.  `keep[d]` (bool (V,) or None) drops hop d = 2mu+s where False."""
    Lx, Ly, Lz, Lt = dims
    V = Lx * Ly * Lz * Lt
    phi = as_field(phi, V)
    L = phi.shape[-1]
    f = phi.reshape(Lt, Lz, Ly, Lx, 4, 3, L)
    U4 = U.reshape(Lt, Lz, Ly, Lx, 4, 3, 3)
    eta = np.zeros_like(f)
    for mu in range(4):
        ax = _axis(mu)
        ph = complex(phases[mu][0], phases[mu][1])
        # forward hop: phi_{x+mu}, phase on the slice x_mu = L_mu - 1
        fw = np.roll(f, -1, axis=ax)
        sl = [slice(None)] * 7
        sl[ax] = -1
        fw[tuple(sl)] *= ph
        hop = _colour(U4[..., mu, :, :], fw)
        hop = _spin(_PM[mu], hop)
        if keep is not None:
            hop *= keep[2 * mu].reshape(Lt, Lz, Ly, Lx)[..., None, None, None]
        eta += hop
        # backward hop: U^dagger_{x-mu} phi_{x-mu}, conj phase on x_mu = 0
        bw = np.roll(f, 1, axis=ax)
        sl = [slice(None)] * 7
        sl[ax] = 0
        bw[tuple(sl)] *= np.conj(ph)
        Ub = np.roll(U4[..., mu, :, :], 1, axis=ax)
        hop = _colour(np.conj(np.swapaxes(Ub, -1, -2)), bw)
        hop = _spin(_PP[mu], hop)
        if keep is not None:
            hop *= keep[2 * mu + 1].reshape(Lt, Lz, Ly, Lx)[..., None, None, None]
        eta += hop
    return eta.reshape(V, 4, 3, L)


def apply_D(U, kappa, phases, phi, dims) -> np.ndarray:
    """A phi = phi - kappa * H phi; returns shape (V, 4, 3, L)."""
    V = int(np.prod(dims))
    phi = as_field(phi, V)
    return phi - kappa * hopping(U, phases, phi, dims)


def domain_keep(dims, block):
    """Per-hop masks keeping only hops whose two ends lie in the same domain."""
    c = geometry.coords(dims)
    keep = []
    for mu in range(4):
        r = c[:, mu] % block[mu]
        keep.append(r != block[mu] - 1)   # forward hop stays inside
        keep.append(r != 0)               # backward hop stays inside
    return keep


def apply_blocked(U, kappa, phases, phi, dims, block) -> np.ndarray:
    """Block-diagonal (Dirichlet) part of A: sum over domains D of A_DD.

    Sec. 2.2 writes A over the two domain colours; A_EE restricted to one
    domain is A with every hop that leaves the domain removed.
    """
    V = int(np.prod(dims))
    phi = as_field(phi, V)
    return phi - kappa * hopping(U, phases, phi, dims, keep=domain_keep(dims, block))


def apply_D_sites(U, kappa, phases, phi, dims, sites) -> np.ndarray:
    """(A phi) at the listed sites only, by an explicit loop over those sites."""
    V = int(np.prod(dims))
    phi = as_field(phi, V)
    L = phi.shape[-1]
    out = np.empty((len(sites), 4, 3, L), dtype=np.complex128)
    for k, s in enumerate(sites):
        s = int(s)
        x = [s % dims[0], (s // dims[0]) % dims[1],
             (s // (dims[0] * dims[1])) % dims[2], s // (dims[0] * dims[1] * dims[2])]
        eta = np.zeros((4, 3, L), dtype=np.complex128)
        for mu in range(4):
            ph = complex(phases[mu][0], phases[mu][1])
            xf = list(x)
            xf[mu] += 1
            fac = 1.0
            if xf[mu] == dims[mu]:
                xf[mu], fac = 0, ph
            sf = int(geometry.site_of(dims, xf))
            eta += np.einsum("st,tal->sal", _PM[mu],
                             np.einsum("ab,tbl->tal", U[s, mu], phi[sf])) * fac
            xb = list(x)
            xb[mu] -= 1
            fac = 1.0
            if xb[mu] < 0:
                xb[mu], fac = dims[mu] - 1, np.conj(ph)
            sb = int(geometry.site_of(dims, xb))
            Ud = np.conj(U[sb, mu]).T
            eta += np.einsum("st,tal->sal", _PP[mu], np.einsum("ab,tbl->tal", Ud, phi[sb])) * fac
        out[k] = phi[s] - kappa * eta
    return out


def dense_D(U, kappa, phases, dims) -> np.ndarray:
    """Explicit N x N matrix of A, assembled one site and one hop at a time.

    Row/column index n = 12*site + 3*spin + colour, so a hop block is
    kron(spin matrix, colour matrix).  Only for tiny lattices.
    """
    V = int(np.prod(dims))
    N = 12 * V
    D = np.zeros((N, N), dtype=np.complex128)
    for s in range(V):
        x = [s % dims[0], (s // dims[0]) % dims[1],
             (s // (dims[0] * dims[1])) % dims[2], s // (dims[0] * dims[1] * dims[2])]
        D[12 * s:12 * s + 12, 12 * s:12 * s + 12] += np.eye(12)
        for mu in range(4):
            ph = complex(phases[mu][0], phases[mu][1])
            xf = list(x)
            xf[mu] += 1
            fac = 1.0
            if xf[mu] == dims[mu]:
                xf[mu], fac = 0, ph
            sf = int(geometry.site_of(dims, xf))
            D[12 * s:12 * s + 12, 12 * sf:12 * sf + 12] -= kappa * fac * np.kron(_PM[mu], U[s, mu])
            xb = list(x)
            xb[mu] -= 1
            fac = 1.0
            if xb[mu] < 0:
                xb[mu], fac = dims[mu] - 1, np.conj(ph)
            sb = int(geometry.site_of(dims, xb))
            D[12 * s:12 * s + 12, 12 * sb:12 * sb + 12] -= \
                kappa * fac * np.kron(_PP[mu], np.conj(U[sb, mu]).T)
    return D


def gamma5_field(phi: np.ndarray) -> np.ndarray:
    """Multiply every site spinor by gamma_5 (spin axis 1)."""
    g5 = _gamma.gamma5()
    return np.einsum("st,vtal->vsal", g5, phi)
