"""SSOR approximate domain inverse B_DD of the SAP preconditioner (Sec. 2.2).

TEST INFRASTRUCTURE ONLY (see the package header).

On one domain the Dirichlet block of A is A_DD = 1 - Lf - Ub, where Lf holds
the forward hops that stay inside the domain,
    (Lf phi)_x = kappa * sum_mu (1 - gamma_mu) U_{x,mu} phi_{x+mu},
and Ub the backward ones,
    (Ub phi)_x = kappa * sum_mu (1 + gamma_mu) U^dagger_{x-mu,mu} phi_{x-mu}
(the paper calls them L_EE and U_EE: "L" is the forward hopping term).  A hop
that stays inside a domain never crosses the lattice boundary, so no boundary
phase enters.

Inverses.  Lf and Ub are nilpotent on a domain: a chain of k forward hops
inside a b_0 x b_1 x b_2 x b_3 block raises the sum of local coordinates by k,
so Lf^k = 0 for k > K = sum_mu (b_mu - 1).  Hence, exactly,
    (1 - w Lf)^{-1} = sum_{k=0}^{K} (w Lf)^k,     and the same for Ub.

The SSOR inverse with N = N_SSOR correction terms and relaxation w:
    B = (1 - w Ub)^{-1} [ sum_{j=0}^{N} (1 - A^S)^j ] (1 - w Lf)^{-1},
    A^S = (1/w) [ (1 - w Lf)^{-1} + (1 - w Ub)^{-1}
                  + (w - 2) (1 - w Lf)^{-1} (1 - w Ub)^{-1} ],
which is (1 - w Lf)^{-1} A_DD (1 - w Ub)^{-1} written without a product with
A_DD (Eisenstat's form), so that B tends to A_DD^{-1} as N grows whenever the
series converges.  The sum is evaluated as c_0 = t, c_j = c_{j-1} - A^S c_{j-1}.

Every operator here is block diagonal over the domains, so one call treats
all domains at once; the SAP domain solve of one colour passes a residual that
vanishes off that colour.
"""

from __future__ import annotations

import numpy as np

from . import clover, dirac


def _keep(dom, forward: bool):
    """Hop masks keeping only the in-domain hops of one direction sense."""
    keep = dirac.domain_keep(dom.dims, dom.block)
    off = np.zeros_like(keep[0])
    return [k if ((d % 2 == 0) == forward) else off for d, k in enumerate(keep)]


def forward_inside(U, kappa, phases, dom, phi, cinv=None):
    """Lf phi: the forward in-domain hops, times kappa (and (1 + T)^{-1} with clover)."""
    phi = dirac.as_field(phi, dom.V)
    h = dirac.hopping(U, phases, phi, dom.dims, keep=_keep(dom, True))
    return kappa * (clover.site_mul(cinv, h) if cinv is not None else h)


def backward_inside(U, kappa, phases, dom, phi, cinv=None):
    """Ub phi: the backward in-domain hops, times kappa (and (1 + T)^{-1} with clover)."""
    phi = dirac.as_field(phi, dom.V)
    h = dirac.hopping(U, phases, phi, dom.dims, keep=_keep(dom, False))
    return kappa * (clover.site_mul(cinv, h) if cinv is not None else h)


def nilpotency_order(block) -> int:
    return int(sum(b - 1 for b in block))


def inv_one_minus(apply, omega, v, K):
    """(1 - omega X)^{-1} v for a nilpotent X (X^{K+1} = 0): sum_k (omega X)^k v."""
    out = v.copy()
    term = v
    for _ in range(K):
        term = omega * apply(term)
        out = out + term
    return out


def ssor_blocked(U, kappa, phases, dom, v, omega: float, nssor: int, cinv=None):
    """B v with B the SSOR inverse of every domain block (N_SSOR = nssor).
    With cinv (clover, Jacobi preconditioned) Lf and Ub carry (1 + T)^{-1},
    which is site-diagonal, so they stay nilpotent."""
    v = dirac.as_field(v, dom.V)
    K = nilpotency_order(dom.block)

    def Finv(x):
        return inv_one_minus(lambda y: forward_inside(U, kappa, phases, dom, y, cinv), omega, x, K)

    def Binv(x):
        return inv_one_minus(lambda y: backward_inside(U, kappa, phases, dom, y, cinv), omega, x, K)

    def A_S(c):
        # the paper's three-term expression
        return (Finv(c) + Binv(c) + (omega - 2.0) * Finv(Binv(c))) / omega

    t = Finv(v)
    c = t
    s = t
    for _ in range(nssor):
        c = c - A_S(c)
        s = s + c
    return Binv(s)


def ssor_domain_solver(U, kappa, phases, dom, omega: float, nssor: int, cinv=None):
    """domain_solve(rho, colour) for `sap.sap`: B_DD on the domains of one colour."""
    def solve(rho, colour):
        return ssor_blocked(U, kappa, phases, dom, rho * dom.mask(colour), omega, nssor, cinv)
    return solve
