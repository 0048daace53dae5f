"""The seeded mesh inputs are valid simplex meshes with nested parent maps."""
import numpy as np
import pytest

import synthmesh as sm


def _volumes(m):
    P = m.coords[m.cells]
    if m.dim == 2:
        a, b = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0]
        return 0.5 * (a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0])
    a, b, c = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]
    return np.einsum("ij,ij->i", np.cross(a, b), c) / 6.0


@pytest.mark.parametrize("make", [
    lambda: sm.annulus(12, 4, jitter=0.15, seed=1, nref=2),
    lambda: sm.box_tets(2, nref=2, jitter=0.1, seed=2, tags={"z0": sm.SLIP}),
    lambda: sm.sphere_shell(8, 4, 2, nref=2, jitter=0.1, seed=1),
])
def test_mesh_is_valid_and_nested(make):
    m = make()
    assert np.all(_volumes(m) > 0)
    # boundary faces are exactly the faces used by one cell
    d = m.dim
    faces = np.concatenate([np.delete(m.cells, k, axis=1) for k in range(d + 1)])
    key, count = np.unique(np.sort(faces, axis=1), axis=0, return_counts=True)
    assert count.max() <= 2
    bkey = np.unique(np.sort(m.bfaces, axis=1), axis=0)
    assert len(bkey) == len(m.bfaces) and np.array_equal(bkey, key[count == 1])
    assert set(np.unique(m.btags)) <= {sm.FARFIELD, sm.SLIP, sm.ISOTHERMAL, sm.ADIABATIC}
    # nested levels: each coarse cell has 2^d children, the volumes add up
    per = 2 ** d
    for l, p in enumerate(m.parents):
        assert np.array_equal(np.bincount(p), np.full(p.max() + 1, per))
    assert m.level_sizes()[-1] * per ** len(m.parents) == m.n_cells


def test_sphere_shell_boundary_on_spheres():
    m = sm.sphere_shell(8, 4, 2, nref=1, jitter=0.1, seed=1, r_in=0.5, r_out=6.0)
    r = np.linalg.norm(m.coords[m.bfaces], axis=2)
    wall = m.btags == sm.SLIP
    np.testing.assert_allclose(r[wall], 0.5, rtol=1e-12)
    np.testing.assert_allclose(r[~wall], 6.0, rtol=1e-12)
