"""Oracle pins for 3-D mixed-element meshes (Sec. 2.2: tetrahedra, pyramids,
prisms and hexahedra with 4, 5, 5 and 6 faces; triangular faces take the
3-point rule, quadrilateral faces a 4-point Gauss rule).

Every expected value comes from closed forms or from an independent
decomposition written here, never from the oracle itself:
* single elements: volume and centroid of a box, a square pyramid, a right
  prism, a square frustum and a tetrahedron, and the area of a trapezoid face;
* the whole frustum-mapped box: total volume 1 + t + t^2/3;
* every cell: the divergence theorem for quadratic vector fields, which ties
  the face normals, areas, Gauss points and weights to the cell's volume
  and centroid;
* the large-stencil reconstruction reproduces a quadratic field exactly when
  fed its exact cell averages (computed here by another tetrahedral split
  and the 10-point vertex/edge-midpoint formula) and its gradients;
* the free stream is preserved; malformed input is rejected.
"""

import numpy as np
import pytest

import synthmesh as sm

# local faces of the input node orders (tetrahedron, pyramid, prism, hexahedron)
FACES = {4: [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)],
         5: [(0, 1, 2, 3), (0, 1, 4), (1, 2, 4), (2, 3, 4), (3, 0, 4)],
         6: [(0, 1, 2), (3, 4, 5), (0, 1, 4, 3), (1, 2, 5, 4), (2, 0, 3, 5)],
         8: [(0, 1, 2, 3), (4, 5, 6, 7), (0, 1, 5, 4), (1, 2, 6, 5), (2, 3, 7, 6), (3, 0, 4, 7)]}


def single(xyz, tag=sm.FARFIELD):
    """A one-cell mixed-element mesh, every face on the far-field boundary."""
    nodes = list(range(len(xyz)))
    bf = [[nodes[a] for a in f] for f in FACES[len(xyz)]]
    return sm.Mesh(3, np.array(xyz, dtype=np.float64), np.array(nodes, dtype=np.int32),
                   np.array([v for f in bf for v in f], dtype=np.int32),
                   np.full(len(bf), tag, dtype=np.int32), [],
                   cell_offsets=np.array([0, len(xyz)], dtype=np.int32),
                   bface_offsets=np.array(np.cumsum([0] + [len(f) for f in bf]), dtype=np.int32))


def geometry(orc, mesh):
    o = orc.Oracle(mesh, n_levels=1, mach=0.5)
    V, Cc = o.cell_geometry(0)
    return o, V, Cc


def test_single_element_volumes_and_centroids(orc):
    a, b, c, h = 1.3, 0.7, 0.9, 1.1
    box = [(0, 0, 0), (a, 0, 0), (a, b, 0), (0, b, 0), (0, 0, c), (a, 0, c), (a, b, c), (0, b, c)]
    _, V, Cc = geometry(orc, single(box))
    assert V[0] == pytest.approx(a * b * c, rel=1e-14)
    np.testing.assert_allclose(Cc[0], [a / 2, b / 2, c / 2], rtol=1e-14)
    pyr = [(0, 0, 0), (a, 0, 0), (a, a, 0), (0, a, 0), (a / 2, a / 2, h)]
    _, V, Cc = geometry(orc, single(pyr))
    assert V[0] == pytest.approx(a * a * h / 3, rel=1e-14)
    np.testing.assert_allclose(Cc[0], [a / 2, a / 2, h / 4], rtol=1e-14)
    pri = [(0, 0, 0), (a, 0, 0), (0, b, 0), (0, 0, c), (a, 0, c), (0, b, c)]
    _, V, Cc = geometry(orc, single(pri))
    assert V[0] == pytest.approx(a * b * c / 2, rel=1e-14)
    np.testing.assert_allclose(Cc[0], [a / 3, b / 3, c / 2], rtol=1e-14)
    s1, s2 = 1.0, 0.6           # square frustum: sides s1 (z = 0) and s2 (z = h), centred on the z axis
    q1 = [(-s1 / 2, -s1 / 2, 0), (s1 / 2, -s1 / 2, 0), (s1 / 2, s1 / 2, 0), (-s1 / 2, s1 / 2, 0)]
    q2 = [(x * s2 / s1, y * s2 / s1, h) for x, y, _ in q1]
    o, V, Cc = geometry(orc, single(q1 + q2))
    A1, A2 = s1 * s1, s2 * s2
    assert V[0] == pytest.approx(h / 3 * (A1 + A2 + np.sqrt(A1 * A2)), rel=1e-14)
    zc = h * (A1 + 2 * np.sqrt(A1 * A2) + 3 * A2) / (4 * (A1 + np.sqrt(A1 * A2) + A2))
    np.testing.assert_allclose(Cc[0], [0, 0, zc], atol=1e-15)
    fg = o.face_geometry(0)
    slant = np.hypot(h, (s1 - s2) / 2)
    side = np.sort(fg["S"])[1:5]          # between the top (s2^2) and the bottom (s1^2)
    np.testing.assert_allclose(side, (s1 + s2) / 2 * slant, rtol=1e-14)   # trapezoid areas
    tet = [(0, 0, 0), (a, 0, 0), (0, b, 0), (0.2, 0.1, c)]
    _, V, Cc = geometry(orc, single(tet))
    assert V[0] == pytest.approx(a * b * c / 6, rel=1e-14)
    np.testing.assert_allclose(Cc[0], np.mean(np.array(tet), axis=0), rtol=1e-14)


@pytest.fixture(scope="module")
def box(orc):
    m = sm.hybrid_box(4, seed=3, taper=0.4)
    return m, orc.Oracle(m, n_levels=3, mach=0.5)


def test_generator_has_every_element_type(box):
    m, _ = box
    for k in ("tets", "pyramids", "prisms", "hexahedra"):
        assert m.info[k] > 0, m.info


def test_total_volume_of_the_frustum_box(box):
    m, o = box
    V, _ = o.cell_geometry(0)
    t = m.info["taper"]
    assert V.sum() == pytest.approx(1.0 + t + t * t / 3.0, rel=1e-13)
    for l in (1, 2):                      # agglomerates keep the volume
        Vl, _ = o.cell_geometry(l)
        assert Vl.sum() == pytest.approx(V.sum(), rel=1e-13)


def test_divergence_theorem_on_every_cell(box):
    """sum over faces of S n . (sum_g w_g F(x_g)) = integral of div F, for
    F = (x^2, y^2, z^2) (div: 2(x + y + z)) and F = (yz, zx, xy) + (x^2, 0, 0)
    (div: 2x): exact for the 3-point triangle and 2 x 2 quadrilateral rules."""
    m, o = box
    V, Cc = o.cell_geometry(0)
    fg = o.face_geometry(0)
    ngp, gp, w = o.face_quadrature()
    assert set(ngp.tolist()) == {3, 4}
    np.testing.assert_allclose(w.sum(axis=1), 1.0, rtol=1e-14)
    # Gauss points lie in the face plane and average to the face centre
    off = np.einsum("fgd,fd->fg", gp - fg["xc"][:, None, :], fg["n"])
    assert np.abs(off[w > 0]).max() < 1e-14
    np.testing.assert_allclose(np.einsum("fg,fgd->fd", w, gp), fg["xc"], atol=1e-14)
    for F, div_avg in ((lambda x: x ** 2, lambda c: 2 * c.sum(axis=1)),
                       (lambda x: np.stack([x[..., 1] * x[..., 2] + x[..., 0] ** 2, x[..., 2] * x[..., 0],
                                            x[..., 0] * x[..., 1]], axis=-1), lambda c: 2 * c[:, 0])):
        flux = fg["S"] * np.einsum("fg,fgd,fd->f", w, F(gp), fg["n"])
        acc = np.zeros(len(V))
        L, R = fg["LR"][:, 0], fg["LR"][:, 1]
        np.add.at(acc, L, flux)
        np.add.at(acc, R[R >= 0], -flux[R >= 0])
        np.testing.assert_allclose(acc, V * div_avg(Cc), rtol=1e-12, atol=1e-15)


def quad_field(x):
    """A quadratic field per conservative component, physical on the unit box."""
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    rho = 1.0 + 0.2 * X - 0.1 * Y + 0.05 * Z + 0.1 * X * X - 0.07 * X * Y + 0.03 * Y * Z + 0.04 * Z * Z
    mx = 0.3 + 0.1 * Y - 0.2 * Z + 0.05 * X * Z - 0.06 * Y * Y
    my = -0.2 + 0.1 * X + 0.08 * X * Y + 0.02 * Z * Z
    mz = 0.1 - 0.05 * X + 0.07 * Y * Z
    E = 3.0 + 0.3 * X * Y - 0.2 * Z + 0.1 * X * X + 0.05 * Y
    return np.stack([rho, mx, my, mz, E], axis=-1)


def quad_grad(x, h=1e-4):
    # central differences are exact for quadratics up to rounding
    g = np.zeros(x.shape[:-1] + (5, 3))
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        g[..., d] = (quad_field(x + e) - quad_field(x - e)) / (2 * h)
    return g


def cell_averages(m):
    """Exact averages of quad_field over every cell: cones from the cell's
    first node to the triangles of the faces not containing it, each
    integrated by the formula V (-1/20 sum of vertex values + 1/5 sum of
    edge-midpoint values), exact for quadratics."""
    X = m.coords
    out = np.zeros((m.n_cells, 5))
    for i in range(m.n_cells):
        nd = m.cells[m.cell_offsets[i]:m.cell_offsets[i + 1]]
        apex = X[nd[0]]
        tot, vol = np.zeros(5), 0.0
        for f in FACES[len(nd)]:
            if 0 in f:
                continue
            cyc = [X[nd[a]] for a in f]
            for t in range(len(cyc) - 2):
                P = np.array([apex, cyc[0], cyc[t + 1], cyc[t + 2]])
                v = abs(np.linalg.det(P[1:] - P[0])) / 6.0
                mids = np.array([(P[a] + P[b]) / 2 for a in range(4) for b in range(a + 1, 4)])
                tot += v * (-quad_field(P).sum(axis=0) / 20.0 + quad_field(mids).sum(axis=0) / 5.0)
                vol += v
        out[i] = tot / vol
    return out


def test_large_stencil_reproduces_quadratics(box):
    m, o = box
    V, Cc = o.cell_geometry(0)
    W = cell_averages(m)
    G = quad_grad(Cc)
    o.set_state(W, G, np.ones(m.n_cells))
    fg = o.face_geometry(0)
    LR = fg["LR"]
    nbrs = np.bincount(LR[LR[:, 1] >= 0].ravel(), minlength=m.n_cells)
    rng = np.random.default_rng(0)
    checked = 0
    for i in np.flatnonzero(nbrs >= 3):
        x = Cc[i] + 0.05 * rng.uniform(-1, 1, size=3) * V[i] ** (1 / 3)
        _, _, p2, _, _ = o.recon_eval(int(i), x)
        np.testing.assert_allclose(p2, quad_field(x), rtol=1e-11, atol=1e-12)
        checked += 1
    assert checked > 0.8 * m.n_cells


def test_free_stream_is_preserved(orc):
    m = sm.hybrid_box(4, seed=5, tags={"z0": sm.SLIP, "z1": sm.SLIP})
    o = orc.Oracle(m, n_levels=3, mach=2.0)
    o.init_freestream()
    R, _, _ = o.residual(0)
    assert np.abs(R).max() < 1e-14


def test_malformed_mixed_input_is_rejected(orc):
    box = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
    bent = [list(p) for p in box]
    bent[6][2] = 1.2                           # the top quadrilateral is no longer planar
    with pytest.raises(RuntimeError, match="non-planar"):
        orc.Oracle(single(bent), n_levels=1, mach=0.5)
    m = single(box)
    m.cell_offsets = np.array([0, 7], dtype=np.int32)
    m.cells = m.cells[:7]
    with pytest.raises(RuntimeError, match="node count"):
        orc.Oracle(m, n_levels=1, mach=0.5)
    m = single(box)
    m.bface_offsets = None
    with pytest.raises(Exception):
        orc.Oracle(m, n_levels=1, mach=0.5)
