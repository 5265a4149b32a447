"""Schwarz alternating procedure (SAP) preconditioner, Sec. 2.2.

With the lattice split into domains coloured E/O (no two domains of one colour
touch), one SAP cycle updates psi on every E domain from the current residual,
then on every O domain from the *updated* residual:

    psi_E += B_EE (eta - A psi)_E ;  psi_O += B_OO (eta - A psi)_O .

Starting from psi = 0, one cycle is psi = K eta with
K = [[B_EE, 0], [-B_OO A_OE B_EE, B_OO]], and each further cycle is
psi <- psi + K (eta - A psi), so ncy cycles give M = K sum_{j<ncy} (1 - A K)^j
(the paper writes the sum to N_SAP; we count ncy applications of K).

B_DD is an approximate inverse of the domain block A_DD.  The paper uses SSOR
(see `ssor`); the default here is the minimal-residual (MR) iteration with a
fixed number of steps, starting from x = 0:
    w = A_DD r ; omega = <w, r> / <w, w> ; x += omega r ; r -= omega w,
one omega per domain and per column (omega = 0 where <w, w> = 0).
"""

from __future__ import annotations

import numpy as np

from . import clover, dirac, geometry


class Domains:
    """Domain bookkeeping for one lattice and block size (from the definitions)."""

    def __init__(self, dims, block):
        geometry.check_domains(dims, block)
        self.dims, self.block = tuple(dims), tuple(block)
        self.V = geometry.volume(dims)
        self.did = geometry.domain_id(dims, block)
        self.colour = geometry.domain_colour(dims, block)
        self.ndom = int(np.prod(geometry.domain_grid(dims, block)))
        self.keep = dirac.domain_keep(dims, block)

    def per_domain_sum(self, vals: np.ndarray) -> np.ndarray:
        """vals (V, L) -> (ndom, L) sums over the sites of each domain."""
        acc = np.zeros((self.ndom,) + vals.shape[1:], dtype=vals.dtype)
        np.add.at(acc, self.did, vals)
        return acc

    def mask(self, colour: int) -> np.ndarray:
        return (self.colour == colour)[:, None, None, None]


def apply_blocked(U, kappa, phases, dom: Domains, phi, cinv=None):
    """A_DD phi on every domain; with cinv = (1 + T)^{-1} per site (clover,
    Jacobi preconditioned) A_DD = 1 - kappa (1 + T)^{-1} H_DD."""
    V = dom.V
    phi = dirac.as_field(phi, V)
    h = dirac.hopping(U, phases, phi, dom.dims, keep=dom.keep)
    if cinv is not None:
        h = clover.site_mul(cinv, h)
    return phi - kappa * h


def apply_A(U, kappa, phases, dims, phi, cinv=None):
    """The full operator: Wilson, or Jacobi-preconditioned clover if cinv is given."""
    if cinv is None:
        return dirac.apply_D(U, kappa, phases, phi, dims)
    return clover.apply_A(U, kappa, phases, cinv, phi, dims)


def mr_domains(U, kappa, phases, dom: Domains, rho, colour: int, nmr: int, cinv=None, trace=None):
    """MR approximation of A_DD^{-1} rho_D on every domain of one colour.

    Each step takes the complex step size that minimises ||r - omega A_DD r||
    on its domain, separately for each column: omega = <w, r> / <w, w> with
    <a, b> = sum conj(a) b.  If `trace` is a list, one record per step is
    appended: the residual norms^2 before and after the step and <w, r_new>,
    each per domain and column (what the MR pins check)."""
    r = dirac.as_field(rho, dom.V) * dom.mask(colour)
    x = np.zeros_like(r)
    for _ in range(nmr):
        w = apply_blocked(U, kappa, phases, dom, r, cinv)
        wr = dom.per_domain_sum(np.sum(np.conj(w) * r, axis=(1, 2)))
        ww = dom.per_domain_sum(np.sum(np.abs(w) ** 2, axis=(1, 2)))
        omega = np.zeros_like(wr)
        nz = ww != 0
        omega[nz] = wr[nz] / ww[nz]
        om = omega[dom.did][:, None, None, :]
        x = x + om * r
        r_new = r - om * w
        if trace is not None:
            trace.append({
                "before": dom.per_domain_sum(np.sum(np.abs(r) ** 2, axis=(1, 2))),
                "after": dom.per_domain_sum(np.sum(np.abs(r_new) ** 2, axis=(1, 2))),
                "w_rnew": dom.per_domain_sum(np.sum(np.conj(w) * r_new, axis=(1, 2))),
                "ww": ww,
                "omega": omega,
            })
        r = r_new
    return x


def sap(U, kappa, phases, dom: Domains, eta, ncy: int, nmr: int, domain_solve=None, cinv=None):
    """psi = M_SAP eta with ncy cycles; domain_solve(rho, colour) -> increment.
    cinv: (1 + T)^{-1} per site for the Jacobi-preconditioned clover operator."""
    if domain_solve is None:
        def domain_solve(rho, colour):
            return mr_domains(U, kappa, phases, dom, rho, colour, nmr, cinv)
    eta = dirac.as_field(eta, dom.V)
    psi = np.zeros_like(eta)
    for _ in range(ncy):
        for colour in (0, 1):
            rho = eta - apply_A(U, kappa, phases, dom.dims, psi, cinv)
            psi = psi + domain_solve(rho * dom.mask(colour), colour)
    return psi


def exact_domain_solver(U, kappa, phases, dom: Domains, cinv=None):
    """domain_solve using dense LU of every A_DD (tiny lattices only)."""
    D = dirac.dense_D(U, kappa, phases, dom.dims)
    if cinv is not None:
        # A = 1 + (1 + T)^{-1} (D_wilson - 1), block-diagonal (1 + T)^{-1}
        N = D.shape[0]
        Cb = np.zeros_like(D)
        for x in range(dom.V):
            Cb[12 * x:12 * x + 12, 12 * x:12 * x + 12] = cinv[x]
        D = np.eye(N) + Cb @ (D - np.eye(N))
    blocks = []
    for d in range(dom.ndom):
        sites = np.nonzero(dom.did == d)[0]
        idx = (12 * sites[:, None] + np.arange(12)[None, :]).ravel()
        blocks.append((d, idx, np.linalg.inv(D[np.ix_(idx, idx)])))

    def solve(rho, colour):
        rho = dirac.as_field(rho, dom.V)
        L = rho.shape[-1]
        flat = rho.reshape(-1, L)
        out = np.zeros_like(flat)
        for d, idx, inv in blocks:
            if dom.colour[dom.did == d][0] == colour:
                out[idx] = inv @ flat[idx]
        return out.reshape(rho.shape)
    return solve
