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


def test_kuhn_shell_counts_nesting_and_boundaries():
    """The survey's C3 shell at a small size: Kuhn tetrahedra of the refined
    index grid minus the polar-degenerate ones (3 of 6 per polar-row cube),
    Freudenthal-nested parents (8 index-space children each), parent-major
    numbering, watertight with the boundary on the two spheres."""
    na, npol, nr, nref = 8, 4, 4, 2
    m = sm.sphere_shell_kuhn(na, npol, nr, nref=nref)
    f = 2 ** nref
    NA, NP, NR = na * f, npol * f, nr * f
    assert m.n_cells == 6 * NA * NP * NR - 2 * 3 * NA * NR
    assert np.all(_volumes(m) > 0)
    faces = np.concatenate([np.delete(m.cells, k, axis=1) for k in range(4)])
    key, count = np.unique(np.sort(faces, axis=1), axis=0, return_counts=True)
    assert count.max() <= 2
    bkey = np.unique(np.sort(m.bfaces, axis=1), axis=0)
    assert len(bkey) == len(m.bfaces) and np.array_equal(bkey, key[count == 1])
    r = np.linalg.norm(m.coords[m.bfaces], axis=2)
    wall = m.btags == sm.SLIP
    np.testing.assert_allclose(r[wall], 0.5, rtol=1e-12)
    np.testing.assert_allclose(r[~wall], 6.0, rtol=1e-12)
    assert wall.sum() == (~wall).sum() == 2 * NA * (NP - 1)   # two triangles per quad, one per pole quad
    # every index-space Kuhn tetrahedron has exactly 8 Kuhn children at twice the resolution
    org, perm = sm._kuhn_tets(2 * na, 2 * npol, 2 * nr)
    po, pp = sm._kuhn_parent(org, perm)
    pk = ((po[:, 0] * npol + po[:, 1]) * nr + po[:, 2]) * 6 + pp
    _, cnt = np.unique(pk, return_counts=True)
    assert len(cnt) == 6 * na * npol * nr and np.all(cnt == 8)
    # parent-major numbering: children of a coarse cell are contiguous, parents ascend
    for p in m.parents:
        assert np.all(np.diff(p) >= 0) and p.max() + 1 == len(np.unique(p))
    # the surviving fine tetrahedra fill the agglomerates: a coarse cell with
    # no degenerate descendants has 8 children
    assert np.bincount(m.parents[0]).max() == 8
