"""Index tables built on the GPU (by the kernels' own index functions) are
bit-exact against the oracle's tables written from their definitions."""

import numpy as np
import pytest

from oracle import geometry

pytestmark = pytest.mark.gpu
gu = pytest.importorskip("tests.gpu_util")


@pytest.mark.parametrize("dims,block", [((4, 4, 4, 4), (2, 2, 2, 2)), ((8, 8, 8, 8), (4, 4, 4, 4)),
                                        ((12, 12, 12, 12), (6, 6, 6, 6)), ((4, 2, 6, 8), (2, 1, 3, 4)),
                                        ((16, 16, 16, 32), (8, 8, 8, 8))])
def test_tables_bit_exact(dims, block):
    gu.flush(f"tables {dims} {block}")
    V = int(np.prod(dims))
    U = np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3)).copy()
    with gu.Lattice(dims, block, U, 0.1) as lat:
        t = lambda name: gu.binding.mbbs_lattice_table(lat.h, name)
        np.testing.assert_array_equal(t("COORD").reshape(V, 4), geometry.coords(dims))
        nb = geometry.neighbours(dims)
        np.testing.assert_array_equal(t("NEIGHBOUR").reshape(V, 8), nb)
        np.testing.assert_array_equal(t("BOUNDARY"), geometry.boundary_flags(dims))
        np.testing.assert_array_equal(t("PARITY"), geometry.parity(dims))
        np.testing.assert_array_equal(t("EO"), geometry.eo_index(dims))
        np.testing.assert_array_equal(t("DOMAIN"), geometry.domain_id(dims, block))
        np.testing.assert_array_equal(t("COLOUR"), geometry.domain_colour(dims, block))
        np.testing.assert_array_equal(t("LOCAL"), geometry.local_index(dims, block))
        dmi = geometry.domain_major_index(dims, block)
        np.testing.assert_array_equal(t("DM_INDEX"), dmi)
        np.testing.assert_array_equal(t("DM_SITE"), geometry.domain_major_site(dims, block))
        np.testing.assert_array_equal(t("LOCAL_NB").reshape(-1, 8), geometry.local_neighbours(block))
        # neighbours in domain-major positions: dmnb[dmi[s]] = dmi[nb[s]]
        dmnb = t("DM_NEIGHBOUR").reshape(V, 8)
        np.testing.assert_array_equal(dmnb[dmi], dmi[nb])
        order, off = geometry.hyperplane_order(block)
        np.testing.assert_array_equal(t("HYPERPLANE"), np.concatenate([order, off]))


def test_create_rejects_bad_geometry():
    V = 4 * 4 * 4 * 6
    U = gu.dev(np.broadcast_to(np.eye(3, dtype=complex), (V, 4, 3, 3)).copy())
    for dims, block in (((4, 4, 4, 6), (2, 2, 2, 2)),     # 3 domains along t
                        ((4, 4, 4, 6), (2, 2, 2, 4))):    # not divisible
        with pytest.raises(gu.binding.MbbsError) as e:
            gu.binding.mbbs_lattice_create(dims, block, U, 0.1, gu.PH_AP)
        assert e.value.code == gu.binding.EINVAL
    with pytest.raises(gu.binding.MbbsError):
        gu.binding.mbbs_lattice_create((4, 4, 4, 6), (2, 2, 2, 3), U, 0.1, ((2.0, 0), (1, 0), (1, 0), (1, 0)))
