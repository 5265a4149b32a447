"""Lattice and SAP-domain index tables, written out from their definitions.

Site order (the paper fixes only N = Lx*Ly*Lz*Lt*12, Sec. 2.1):
  site = x + Lx*(y + Ly*(z + Lz*t)), mu = 0,1,2,3 is x,y,z,t.
Hop index d = 2*mu + s, s = 0 forward (site + mu), s = 1 backward (site - mu).

SAP domains (Sec. 2.2: the lattice is split into domains coloured even/odd,
A is written as the 2x2 block matrix over the two colours): with block
(bx,by,bz,bt), the domain coordinate is x_mu div b_mu, the domain id is
lexicographic over the domain grid, the colour is the parity of the sum of
domain coordinates (colour 0 = "E" is swept first), the local index is
lexicographic over x_mu mod b_mu.  Domain-major order lists all colour-0
domains in id order, then all colour-1 domains, each with its local sites.

Site parity / even-odd index: parity = (x+y+z+t) mod 2, eo = parity*V/2 +
site//2 (valid since Lx is even).
"""

from __future__ import annotations

import numpy as np


def volume(dims) -> int:
    return int(np.prod(dims))


def coords(dims) -> np.ndarray:
    """(V, 4) int64 coordinates (x, y, z, t) of every site."""
    Lx, Ly, Lz, Lt = dims
    s = np.arange(volume(dims), dtype=np.int64)
    return np.stack([s % Lx, (s // Lx) % Ly, (s // (Lx * Ly)) % Lz,
                     s // (Lx * Ly * Lz)], axis=1)


def site_of(dims, c) -> np.ndarray:
    Lx, Ly, Lz, _ = dims
    c = np.asarray(c)
    return c[..., 0] + Lx * (c[..., 1] + Ly * (c[..., 2] + Lz * c[..., 3]))


def neighbours(dims) -> np.ndarray:
    """(V, 8): column 2mu is site+mu, column 2mu+1 is site-mu (periodic wrap)."""
    c = coords(dims)
    out = np.empty((c.shape[0], 8), dtype=np.int64)
    for mu in range(4):
        for s, step in ((0, 1), (1, -1)):
            d = c.copy()
            d[:, mu] = (d[:, mu] + step) % dims[mu]
            out[:, 2 * mu + s] = site_of(dims, d)
    return out


def boundary_flags(dims) -> np.ndarray:
    """(V,) bit 2mu+s set when hop (mu, s) crosses the lattice boundary."""
    c = coords(dims)
    f = np.zeros(c.shape[0], dtype=np.int64)
    for mu in range(4):
        f |= (c[:, mu] == dims[mu] - 1).astype(np.int64) << (2 * mu)
        f |= (c[:, mu] == 0).astype(np.int64) << (2 * mu + 1)
    return f


def parity(dims) -> np.ndarray:
    return coords(dims).sum(axis=1) % 2


def eo_index(dims) -> np.ndarray:
    V = volume(dims)
    return parity(dims) * (V // 2) + np.arange(V) // 2


def domain_grid(dims, block) -> tuple:
    return tuple(d // b for d, b in zip(dims, block))


def domain_id(dims, block) -> np.ndarray:
    c = coords(dims)
    nd = domain_grid(dims, block)
    dc = c // np.asarray(block)
    return dc[:, 0] + nd[0] * (dc[:, 1] + nd[1] * (dc[:, 2] + nd[2] * dc[:, 3]))


def domain_colour(dims, block) -> np.ndarray:
    c = coords(dims)
    return (c // np.asarray(block)).sum(axis=1) % 2


def local_index(dims, block) -> np.ndarray:
    c = coords(dims) % np.asarray(block)
    bx, by, bz, _ = block
    return c[:, 0] + bx * (c[:, 1] + by * (c[:, 2] + bz * c[:, 3]))


def domain_major_site(dims, block) -> np.ndarray:
    """(V,) lexicographic site at each position of domain-major order."""
    nd = domain_grid(dims, block)
    ndom = int(np.prod(nd))
    Vb = int(np.prod(block))
    d = np.arange(ndom)
    dcoord = np.stack([d % nd[0], (d // nd[0]) % nd[1],
                       (d // (nd[0] * nd[1])) % nd[2], d // (nd[0] * nd[1] * nd[2])], 1)
    dcol = dcoord.sum(axis=1) % 2
    order_dom = np.concatenate([d[dcol == 0], d[dcol == 1]])
    rank = np.empty(ndom, dtype=np.int64)
    rank[order_dom] = np.arange(ndom)
    pos = rank[domain_id(dims, block)] * Vb + local_index(dims, block)
    out = np.empty_like(pos)
    out[pos] = np.arange(pos.size)
    return out


def domain_major_index(dims, block) -> np.ndarray:
    """(V,) position of each lexicographic site in domain-major order."""
    dm = domain_major_site(dims, block)
    out = np.empty_like(dm)
    out[dm] = np.arange(dm.size)
    return out


def local_neighbours(block) -> np.ndarray:
    """(Vb, 8) in-domain neighbour (local index) per hop, -1 if it leaves."""
    bx, by, bz, bt = block
    Vb = bx * by * bz * bt
    l = np.arange(Vb)
    c = np.stack([l % bx, (l // bx) % by, (l // (bx * by)) % bz, l // (bx * by * bz)], 1)
    out = np.empty((Vb, 8), dtype=np.int64)
    for mu in range(4):
        for s, step in ((0, 1), (1, -1)):
            d = c.copy()
            d[:, mu] += step
            inside = (d[:, mu] >= 0) & (d[:, mu] < block[mu])
            li = d[:, 0] + bx * (d[:, 1] + by * (d[:, 2] + bz * d[:, 3]))
            out[:, 2 * mu + s] = np.where(inside, li, -1)
    return out


def hyperplane_order(block):
    """SSOR wavefront order inside a domain: local indices sorted by the
    hyperplane h = l_0 + l_1 + l_2 + l_3 (ties by local index), and the
    offsets of h = 0 .. H (H = sum_mu (b_mu - 1)).  A forward hop raises h by
    one, so sites of one hyperplane never depend on each other in a
    triangular sweep."""
    bx, by, bz, bt = block
    Vb = bx * by * bz * bt
    l = np.arange(Vb)
    h = l % bx + (l // bx) % by + (l // (bx * by)) % bz + l // (bx * by * bz)
    order = np.argsort(h, kind="stable")
    nh = sum(b - 1 for b in block) + 1
    off = np.concatenate([[0], np.cumsum(np.bincount(h, minlength=nh))])
    return order, off


def check_domains(dims, block) -> None:
    """Raise ValueError unless every extent is even and 2-colourable by domains."""
    for d, b in zip(dims, block):
        if d <= 0 or d % 2 or b <= 0 or d % b:
            raise ValueError(f"extent {d} not even or not divisible by block {b}")
        if (d // b) % 2:
            raise ValueError(f"{d // b} domains along a direction: not 2-colourable")
