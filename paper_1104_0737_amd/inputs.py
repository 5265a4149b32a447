"""Seeded synthetic inputs: SU(3) gauge fields and right-hand-side blocks.

This module only *draws* inputs.  It holds none of the solver's arithmetic
(no Dirac operator, no Schwarz preconditioner, no Krylov step), so that the
CPU oracle tests and the GPU path can share identical inputs without sharing
any of the method's code.

Conventions (the paper fixes none of them; its problem statement is in
Sec. 2.1, where N = Lx*Ly*Lz*Lt*3*4 and X, B are N x L):

* site = x + Lx*(y + Ly*(z + Lz*t)), direction mu = 0,1,2,3 is x,y,z,t.
* A spinor block is complex128 of shape (N, L), row n = 12*site + 3*spin +
  colour, right-hand side i fastest in memory (Sec. 2.1, "i running first").
* A gauge field is complex128 of shape (V, 4, 3, 3): U[site, mu, a, b] is the
  link from site to site + mu (Eq. for the hopping term).

Gauge links are U = exp(i*eps*H), H Hermitian traceless with N(0,1) entries,
then re-unitarised.  Draw order per site (lexicographic) and per mu: three
diagonal reals, then Re and Im of the (0,1), (0,2), (1,2) entries.
"""

from __future__ import annotations

import numpy as np

_OFFDIAG = ((0, 1), (0, 2), (1, 2))


def _su3_from_normals(g: np.ndarray, eps: float) -> np.ndarray:
    """Map rows of 9 normals to SU(3) matrices exp(i eps H), re-unitarised."""
    n = g.shape[0]
    H = np.zeros((n, 3, 3), dtype=np.complex128)
    for a in range(3):
        H[:, a, a] = g[:, a]
    for k, (i, j) in enumerate(_OFFDIAG):
        z = g[:, 3 + 2 * k] + 1j * g[:, 4 + 2 * k]
        H[:, i, j] = z
        H[:, j, i] = np.conj(z)
    tr = (H[:, 0, 0] + H[:, 1, 1] + H[:, 2, 2]) / 3.0
    for a in range(3):
        H[:, a, a] -= tr
    w, v = np.linalg.eigh(H)
    U = (v * np.exp(1j * eps * w)[:, None, :]) @ np.conj(np.swapaxes(v, 1, 2))
    # re-unitarise: normalise row 0, orthogonalise row 1, row 2 = conj(r0 x r1)
    r0 = U[:, 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=1)[:, None]
    r1 = U[:, 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=1)[:, None] * r0
    r1 = r1 / np.linalg.norm(r1, axis=1)[:, None]
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=1)


def gauge_field(dims, eps: float, seed: int, chunk: int = 1 << 19) -> np.ndarray:
    """Random SU(3) field of shape (V, 4, 3, 3), drawn in chunks (same stream)."""
    V = int(np.prod(dims))
    rng = np.random.default_rng(seed)
    out = np.empty((V * 4, 3, 3), dtype=np.complex128)
    for s in range(0, V * 4, chunk):
        e = min(V * 4, s + chunk)
        out[s:e] = _su3_from_normals(rng.standard_normal((e - s, 9)), eps)
    return out.reshape(V, 4, 3, 3)


def point_sources(V: int, L: int, site: int, comp0: int = 0) -> np.ndarray:
    """Column j is the unit vector at (site, spin-colour component comp0 + j)."""
    if comp0 + L > 12:
        raise ValueError("point sources cover at most 12 spin-colour components")
    B = np.zeros((12 * V, L), dtype=np.complex128)
    for j in range(L):
        B[12 * site + comp0 + j, j] = 1.0
    return B


def z2_sources(V: int, L: int, seed: int) -> np.ndarray:
    """Every complex entry is +1 or -1 (imaginary part 0) with probability 1/2."""
    rng = np.random.default_rng(seed)
    return (rng.integers(0, 2, size=(12 * V, L)) * 2 - 1).astype(np.complex128)


def gaussian_block(V: int, L: int, seed: int) -> np.ndarray:
    """Complex Gaussian block (unit variance per real component)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((12 * V, L)) + 1j * rng.standard_normal((12 * V, L))


def source_site(V: int, seed: int) -> int:
    """Seeded source position."""
    return int(np.random.default_rng(seed).integers(V))


def random_su3(n: int, seed: int, eps: float = 1.0) -> np.ndarray:
    """n random SU(3) matrices (for gauge transformations in tests)."""
    rng = np.random.default_rng(seed)
    return _su3_from_normals(rng.standard_normal((n, 9)), eps)
