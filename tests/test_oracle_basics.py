"""Pins of the oracle's gamma basis, index tables and gauge inputs.

Each check compares against something other than the oracle's own formula:
the Clifford algebra, brute-force loops over tiny lattices, and group
properties of SU(3).
"""

import itertools

import numpy as np
import pytest

from oracle import gamma, geometry
from paper_1104_0737_amd import inputs


def test_clifford_and_hermiticity():
    g = gamma.gammas()
    for m, n in itertools.product(range(4), repeat=2):
        np.testing.assert_allclose(g[m] @ g[n] + g[n] @ g[m], 2.0 * (m == n) * np.eye(4), atol=0)
    for m in range(4):
        np.testing.assert_allclose(g[m], g[m].conj().T, atol=0)
    np.testing.assert_allclose(gamma.gamma5(), np.diag([1, 1, -1, -1]), atol=0)


def test_projectors_rank_two():
    pm, pp = gamma.projectors()
    for mu in range(4):
        # (1 -/+ gamma)/2 are complementary orthogonal projectors of rank 2
        a, b = pm[mu] / 2, pp[mu] / 2
        np.testing.assert_allclose(a @ a, a, atol=1e-15)
        np.testing.assert_allclose(a @ b, 0, atol=1e-15)
        assert np.linalg.matrix_rank(pm[mu]) == 2


def _brute_tables(dims, block):
    """All tables from the definitions, by plain Python loops."""
    Lx, Ly, Lz, Lt = dims
    V = Lx * Ly * Lz * Lt
    nd = [d // b for d, b in zip(dims, block)]
    Vb = block[0] * block[1] * block[2] * block[3]
    sites = {}
    for t in range(Lt):
        for z in range(Lz):
            for y in range(Ly):
                for x in range(Lx):
                    sites[(x, y, z, t)] = len(sites)
    coord = {s: c for c, s in sites.items()}
    nb = np.zeros((V, 8), int)
    flags = np.zeros(V, int)
    par = np.zeros(V, int)
    did = np.zeros(V, int)
    col = np.zeros(V, int)
    loc = np.zeros(V, int)
    for s in range(V):
        c = coord[s]
        for mu in range(4):
            f = list(c)
            f[mu] = (f[mu] + 1) % dims[mu]
            b = list(c)
            b[mu] = (b[mu] - 1) % dims[mu]
            nb[s, 2 * mu] = sites[tuple(f)]
            nb[s, 2 * mu + 1] = sites[tuple(b)]
            if c[mu] == dims[mu] - 1:
                flags[s] |= 1 << (2 * mu)
            if c[mu] == 0:
                flags[s] |= 1 << (2 * mu + 1)
        par[s] = sum(c) % 2
        dc = [c[m] // block[m] for m in range(4)]
        did[s] = dc[0] + nd[0] * (dc[1] + nd[1] * (dc[2] + nd[2] * dc[3]))
        col[s] = sum(dc) % 2
        lc = [c[m] % block[m] for m in range(4)]
        loc[s] = lc[0] + block[0] * (lc[1] + block[1] * (lc[2] + block[2] * lc[3]))
    # even/odd: sites of each parity in increasing site order
    eo = np.zeros(V, int)
    k = [0, 0]
    for s in range(V):
        eo[s] = par[s] * (V // 2) + k[par[s]]
        k[par[s]] += 1
    # domain-major: colour-0 domains by id, then colour-1; local order inside
    doms = sorted(set(did.tolist()), key=lambda d: (col[did == d][0], d))
    dm_site = []
    for d in doms:
        members = sorted([s for s in range(V) if did[s] == d], key=lambda s: loc[s])
        dm_site.extend(members)
    lnb = np.zeros((Vb, 8), int)
    for l in range(Vb):
        lc = [l % block[0], (l // block[0]) % block[1],
              (l // (block[0] * block[1])) % block[2], l // (block[0] * block[1] * block[2])]
        for mu in range(4):
            for sgn, step in ((0, 1), (1, -1)):
                q = list(lc)
                q[mu] += step
                if 0 <= q[mu] < block[mu]:
                    lnb[l, 2 * mu + sgn] = q[0] + block[0] * (q[1] + block[1] * (q[2] + block[2] * q[3]))
                else:
                    lnb[l, 2 * mu + sgn] = -1
    return dict(coords=np.array([coord[s] for s in range(V)]), nb=nb, flags=flags, parity=par,
                eo=eo, did=did, colour=col, local=loc, dm_site=np.array(dm_site), lnb=lnb)


@pytest.mark.parametrize("dims,block", [((2, 2, 2, 2), (1, 1, 1, 1)),
                                        ((4, 4, 4, 4), (2, 2, 2, 2)),
                                        ((4, 2, 6, 8), (2, 1, 3, 4)),
                                        ((8, 4, 4, 4), (4, 2, 2, 2))])
def test_tables_brute_force(dims, block):
    b = _brute_tables(dims, block)
    np.testing.assert_array_equal(geometry.coords(dims), b["coords"])
    np.testing.assert_array_equal(geometry.neighbours(dims), b["nb"])
    np.testing.assert_array_equal(geometry.boundary_flags(dims), b["flags"])
    np.testing.assert_array_equal(geometry.parity(dims), b["parity"])
    np.testing.assert_array_equal(geometry.eo_index(dims), b["eo"])
    np.testing.assert_array_equal(geometry.domain_id(dims, block), b["did"])
    np.testing.assert_array_equal(geometry.domain_colour(dims, block), b["colour"])
    np.testing.assert_array_equal(geometry.local_index(dims, block), b["local"])
    np.testing.assert_array_equal(geometry.domain_major_site(dims, block), b["dm_site"])
    np.testing.assert_array_equal(geometry.local_neighbours(block), b["lnb"])


@pytest.mark.parametrize("dims,block", [((4, 4, 4, 4), (2, 2, 2, 2)), ((8, 8, 4, 4), (4, 4, 2, 2))])
def test_table_invariants(dims, block):
    V = geometry.volume(dims)
    nb = geometry.neighbours(dims)
    par = geometry.parity(dims)
    for mu in range(4):
        np.testing.assert_array_equal(nb[nb[:, 2 * mu], 2 * mu + 1], np.arange(V))
        assert np.all(par[nb[:, 2 * mu]] != par)           # every hop flips parity
    assert np.sum(par == 0) == V // 2
    eo = geometry.eo_index(dims)
    assert sorted(eo.tolist()) == list(range(V))
    did = geometry.domain_id(dims, block)
    col = geometry.domain_colour(dims, block)
    Vb = int(np.prod(block))
    assert np.all(np.bincount(did) == Vb)                   # each site in exactly one domain
    assert np.sum(col == 0) == V // 2
    for d in range(8):                                      # neighbouring domains differ in colour
        cross = did[nb[:, d]] != did
        assert np.all(col[nb[cross, d]] != col[cross])
    dm = geometry.domain_major_site(dims, block)
    assert sorted(dm.tolist()) == list(range(V))
    dmi = geometry.domain_major_index(dims, block)
    np.testing.assert_array_equal(dmi[dm], np.arange(V))


def test_two_domains_per_direction_share_neighbour():
    # with two domains along x, domain 0 meets domain 1 across both its x faces
    dims, block = (4, 4, 4, 4), (2, 2, 2, 2)
    did = geometry.domain_id(dims, block)
    nb = geometry.neighbours(dims)
    c = geometry.coords(dims)
    s_hi = geometry.site_of(dims, [1, 0, 0, 0])   # forward face of domain 0
    s_lo = geometry.site_of(dims, [0, 0, 0, 0])   # backward face of domain 0
    assert did[s_hi] == did[s_lo] == 0
    assert did[nb[s_hi, 0]] == did[nb[s_lo, 1]] == 1
    assert c[nb[s_lo, 1], 0] == 3                  # reached through the wrap


def test_domain_checks():
    geometry.check_domains((8, 8, 8, 8), (4, 4, 4, 4))
    with pytest.raises(ValueError):
        geometry.check_domains((8, 8, 8, 12), (4, 4, 4, 4))   # 3 domains
    with pytest.raises(ValueError):
        geometry.check_domains((8, 8, 8, 9), (4, 4, 4, 3))    # odd extent


def test_gauge_links_su3_and_reproducible():
    U = inputs.gauge_field((2, 2, 2, 4), 0.3, 11)
    m = U.reshape(-1, 3, 3)
    np.testing.assert_allclose(m @ np.conj(np.swapaxes(m, 1, 2)), np.broadcast_to(np.eye(3), m.shape),
                               atol=1e-15)
    np.testing.assert_allclose(np.linalg.det(m), 1.0, atol=1e-15)
    U2 = inputs.gauge_field((2, 2, 2, 4), 0.3, 11, chunk=7)
    assert U.tobytes() == U2.tobytes()
    # eps -> 0 gives the unit field; eps scales the distance from 1
    U0 = inputs.gauge_field((2, 2, 2, 2), 1e-9, 3)
    np.testing.assert_allclose(U0, np.broadcast_to(np.eye(3), U0.shape), atol=1e-8)


def test_gauge_matches_exponential_series():
    # exp(i eps H) from eigh agrees with a Taylor series of the same H
    rng = np.random.default_rng(5)
    g = rng.standard_normal((4, 9))
    U = inputs._su3_from_normals(g, 0.3)
    for k in range(4):
        H = np.zeros((3, 3), complex)
        H[[0, 1, 2], [0, 1, 2]] = g[k, :3]
        for j, (a, b) in enumerate(((0, 1), (0, 2), (1, 2))):
            H[a, b] = g[k, 3 + 2 * j] + 1j * g[k, 4 + 2 * j]
            H[b, a] = np.conj(H[a, b])
        H -= np.trace(H) / 3 * np.eye(3)
        E, term = np.eye(3, dtype=complex), np.eye(3, dtype=complex)
        for n in range(1, 40):
            term = term @ (1j * 0.3 * H) / n
            E = E + term
        np.testing.assert_allclose(U[k], E, atol=1e-13)


def test_sources():
    B = inputs.point_sources(16, 4, 3, 2)
    assert B.shape == (192, 4)
    for j in range(4):
        assert B[12 * 3 + 2 + j, j] == 1 and np.count_nonzero(B[:, j]) == 1
    Z = inputs.z2_sources(16, 3, 9)
    assert set(np.unique(Z).tolist()) <= {-1, 1}
    assert np.all(Z.imag == 0)
