"""Pins of the direct slope evolution (Sec. 2.4) and of the pieces of the
nonlinear reconstruction (Sec. 3): the Green-Gauss sub-stencil, the
smoothness indicators and the nonlinear weights.

* Slope evolution: for continuous linear data the interface distribution at
  t -> 0 is the Maxwellian of the data at the Gauss point, so the evolved
  slope (1/V) sum_f S_f sum_k w_k W(x_fk, dt) n_f tends to the exact gradient
  as dt -> 0 (the face rule is exact for linear W).  Checked on interior cells
  in 2-D and 3-D and on cells with slip-wall faces (data with zero normal
  momentum, so that the mirror ghost continues the data).
* Green-Gauss p^1: exact for linear data when every interior face's midpoint
  is the midpoint of the two cell centroids, which holds on a uniform
  triangulation where each pair of neighbours forms a parallelogram.
* beta_0 of p^2 against the exact integrals of the squared derivatives of a
  reproduced quadratic (closed-form triangle moments); beta_0 = beta_1 on
  linear data on the uniform triangulation, so the weights equal the linear
  weights and the combined polynomial is p^2.
"""
import numpy as np
import pytest

import synthmesh as sm

G = 1.4


def _cells_without(fg, n_cells, tags_excluded):
    """Cells with no boundary face of the given tags (all boundary faces if None)."""
    bad = np.zeros(n_cells, dtype=bool)
    LR, tag = fg["LR"], fg["tag"]
    for f in range(len(LR)):
        if LR[f, 1] < 0 and (tags_excluded is None or tag[f] in tags_excluded):
            bad[LR[f, 0]] = True
    return np.where(~bad)[0]


def _linear_cons(C, c0, A):
    """Conservative state whose every component is linear: W_q = c0_q + A_q . x."""
    return c0[None, :] + C @ A.T


def _retag(mesh, axis_values, tag):
    """Copy of a box/square mesh with the boundary faces on the planes x_axis = value retagged."""
    bt = mesh.btags.copy()
    for f, nodes in enumerate(mesh.bfaces):
        c = mesh.coords[nodes]
        for ax, val in axis_values:
            if np.all(np.abs(c[:, ax] - val) < 1e-12):
                bt[f] = tag
    return sm.Mesh(mesh.dim, mesh.coords, mesh.cells, mesh.bfaces, bt, mesh.parents, dict(mesh.info))


def _evolved_slope_error(orc, mesh, W, A, keep_tags, **kw):
    o = orc.Oracle(mesh, n_levels=1, weno_gamma_large=1.0, cfl_exp=1e-8, **kw)
    grad = np.broadcast_to(A, (mesh.n_cells,) + A.shape).copy()
    o.set_state(W, grad)
    _, gnew, anew = o.residual(0)
    cells = _cells_without(o.face_geometry(0), mesh.n_cells, keep_tags)
    assert len(cells) > 0
    assert np.all(anew[cells] == 1.0)
    return np.abs(gnew[cells] - A[None]).max() / np.abs(A).max()


@pytest.mark.parametrize("reynolds", [0.0, 200.0])
def test_evolved_slope_of_linear_data_2d(orc, reynolds):
    mesh = sm.structured_square(6, jitter=0.25, seed=2, tag=sm.FARFIELD)
    o = orc.Oracle(mesh, n_levels=1)
    _, C = o.cell_geometry(0)
    c0 = np.array([1.0, 0.3, 0.05, 1.0 / (G * (G - 1)) + 0.05])
    A = np.array([[0.04, -0.03], [0.02, 0.05], [-0.03, 0.01], [0.06, 0.02]])
    err = _evolved_slope_error(orc, mesh, _linear_cons(C, c0, A), A, None, mach=0.3, reynolds=reynolds)
    assert err < 1e-8, err


def test_evolved_slope_of_linear_data_3d(orc):
    mesh = sm.box_tets(2, nref=1, jitter=0.1, seed=3)
    o = orc.Oracle(mesh, n_levels=1, dim=3)
    _, C = o.cell_geometry(0)
    c0 = np.array([1.0, 0.3, 0.05, -0.02, 1.0 / (G * (G - 1)) + 0.05])
    A = np.array([[0.04, -0.03, 0.01], [0.02, 0.05, -0.01], [-0.03, 0.01, 0.02],
                  [0.01, -0.02, 0.03], [0.06, 0.02, -0.04]])
    err = _evolved_slope_error(orc, mesh, _linear_cons(C, c0, A), A, None, dim=3, mach=0.3)
    assert err < 1e-8, err


def test_evolved_slope_at_slip_walls_2d(orc):
    """Slip walls on y = 0 and y = 1 (far field on the x sides): cells with wall
    faces included; the normal momentum vanishes, the rest is linear."""
    mesh = _retag(sm.structured_square(6, jitter=0.25, seed=5, tag=sm.SLIP), [(0, 0.0), (0, 1.0)],
                  sm.FARFIELD)
    o = orc.Oracle(mesh, n_levels=1)
    _, C = o.cell_geometry(0)
    c0 = np.array([1.0, 0.3, 0.0, 1.0 / (G * (G - 1)) + 0.05])
    A = np.array([[0.04, -0.03], [0.02, 0.05], [0.0, 0.0], [0.06, 0.02]])
    fg = o.face_geometry(0)
    walls = {int(fg["LR"][f, 0]) for f in range(len(fg["S"])) if fg["LR"][f, 1] < 0 and fg["tag"][f] == sm.SLIP}
    kept = set(_cells_without(fg, mesh.n_cells, (sm.FARFIELD,)).tolist())
    assert len(walls & kept) >= 6
    err = _evolved_slope_error(orc, mesh, _linear_cons(C, c0, A), A, (sm.FARFIELD,), mach=0.3)
    assert err < 1e-8, err


def test_evolved_slope_at_slip_walls_3d(orc):
    mesh = sm.box_tets(2, nref=1, jitter=0.1, seed=4, tags={"z0": sm.SLIP, "z1": sm.SLIP})
    o = orc.Oracle(mesh, n_levels=1, dim=3)
    _, C = o.cell_geometry(0)
    c0 = np.array([1.0, 0.3, 0.05, 0.0, 1.0 / (G * (G - 1)) + 0.05])
    A = np.array([[0.04, -0.03, 0.01], [0.02, 0.05, -0.01], [-0.03, 0.01, 0.02],
                  [0.0, 0.0, 0.0], [0.06, 0.02, -0.04]])
    err = _evolved_slope_error(orc, mesh, _linear_cons(C, c0, A), A, (sm.FARFIELD,), dim=3, mach=0.3)
    assert err < 1e-8, err


def test_evolved_slope_detects_time_evolution(orc):
    """Control: at a finite explicit time step the evolved slope of the same data
    differs from the data's gradient (the pin above is not vacuous)."""
    mesh = sm.structured_square(6, jitter=0.25, seed=2, tag=sm.FARFIELD)
    o = orc.Oracle(mesh, n_levels=1, weno_gamma_large=1.0, cfl_exp=0.5, mach=0.3)
    _, C = o.cell_geometry(0)
    c0 = np.array([1.0, 0.3, 0.05, 1.0 / (G * (G - 1)) + 0.05])
    A = np.array([[0.04, -0.03], [0.02, 0.05], [-0.03, 0.01], [0.06, 0.02]])
    o.set_state(_linear_cons(C, c0, A), np.broadcast_to(A, (mesh.n_cells, 4, 2)).copy())
    _, gnew, _ = o.residual(0)
    cells = _cells_without(o.face_geometry(0), mesh.n_cells, None)
    assert np.abs(gnew[cells] - A[None]).max() / np.abs(A).max() > 1e-6


def _uniform_linear(orc, alpha=None):
    mesh = sm.structured_square(6, jitter=0.0, tag=sm.FARFIELD)
    o = orc.Oracle(mesh, n_levels=1, mach=0.3)
    V, C = o.cell_geometry(0)
    c0 = np.array([1.0, 0.3, 0.05, 1.0 / (G * (G - 1)) + 0.05])
    A = np.array([[0.04, -0.03], [0.02, 0.05], [-0.03, 0.01], [0.06, 0.02]])
    o.set_state(_linear_cons(C, c0, A), np.broadcast_to(A, (mesh.n_cells, 4, 2)).copy(), alpha)
    cells = _cells_without(o.face_geometry(0), mesh.n_cells, None)
    return o, mesh, V, C, A, cells


def test_green_gauss_exact_on_uniform_triangulation(orc):
    o, mesh, V, C, A, cells = _uniform_linear(orc)
    assert len(cells) >= 30
    for i in cells:
        _, _, g1, _ = o.recon_indicators(int(i))
        np.testing.assert_allclose(g1, A, rtol=0, atol=1e-13)


def test_green_gauss_scaled_by_stored_df(orc):
    alpha = np.full(72, 0.37)
    o, mesh, V, C, A, cells = _uniform_linear(orc, alpha)
    for i in cells[:10]:
        _, _, g1, _ = o.recon_indicators(int(i))
        np.testing.assert_allclose(g1, 0.37 * A, rtol=0, atol=1e-13)


def test_equal_indicators_give_linear_weights_and_p2(orc):
    """Linear data on the uniform triangulation: p^2 and p^1 are the same linear
    function, beta_0 = beta_1 = V |A_q|^2, the weights are the linear weights
    and the combined polynomial is p^2 (= the data)."""
    o, mesh, V, C, A, cells = _uniform_linear(orc)
    c0 = np.array([1.0, 0.3, 0.05, 1.0 / (G * (G - 1)) + 0.05])
    for i in cells:
        b0, b1, _, w = o.recon_indicators(int(i))
        np.testing.assert_allclose(b0, V[i] * (A ** 2).sum(axis=1), rtol=1e-12)
        np.testing.assert_allclose(b1, b0, rtol=1e-12)
        np.testing.assert_allclose(w, 0.95, rtol=1e-13)
        x = C[i] + np.array([0.02, -0.01])
        Wx, gx, p2, p1, _ = o.recon_eval(int(i), x)
        np.testing.assert_allclose(Wx, c0 + A @ x, rtol=0, atol=1e-14)
        np.testing.assert_allclose(p2, c0 + A @ x, rtol=0, atol=1e-14)
        np.testing.assert_allclose(gx, A, rtol=0, atol=1e-12)


def _tri_avg_quadratic(P, c):
    """Exact average over triangles P [n,3,2] of c0 + c1 x + c2 y + c3 x^2 + c4 xy + c5 y^2."""
    x0, x1, x2 = P[:, 0, 0], P[:, 1, 0], P[:, 2, 0]
    y0, y1, y2 = P[:, 0, 1], P[:, 1, 1], P[:, 2, 1]
    ax, ay = (x0 + x1 + x2) / 3, (y0 + y1 + y2) / 3
    axx = (x0 * x0 + x1 * x1 + x2 * x2 + x0 * x1 + x1 * x2 + x2 * x0) / 6
    ayy = (y0 * y0 + y1 * y1 + y2 * y2 + y0 * y1 + y1 * y2 + y2 * y0) / 6
    axy = (2 * (x0 * y0 + x1 * y1 + x2 * y2) + x0 * y1 + x1 * y0 + x1 * y2 + x2 * y1 + x2 * y0 + x0 * y2) / 12
    return c[0] + c[1] * ax + c[2] * ay + c[3] * axx + c[4] * axy + c[5] * ayy


def _square_linear(a, b, c):
    """(a + b x + c y)^2 as quadratic coefficients (1, x, y, x^2, xy, y^2)."""
    return np.array([a * a, 2 * a * b, 2 * a * c, b * b, 2 * b * c, c * c])


def test_beta0_is_the_integral_of_squared_derivatives(orc):
    """Sec. 3 indicator of the large stencil: for reproduced quadratic data
    beta_0 = int (q_x^2 + q_y^2) dV + V^2 (q_xx^2 + q_xy^2 + q_yy^2) in 2-D."""
    m = sm.annulus(12, 4, jitter=0.15, seed=9, nref=1, wall_tag=sm.FARFIELD)
    o = orc.Oracle(m, n_levels=1, mach=0.3)
    V, C = o.cell_geometry(0)
    coefs = [np.array([1.0, 0.01, -0.02, 0.003, 0.002, -0.001]),
             np.array([0.3, 0.02, 0.01, -0.002, 0.001, 0.003]),
             np.array([-0.1, 0.01, 0.02, 0.001, -0.003, 0.002]),
             np.array([2.0, -0.03, 0.01, 0.002, 0.001, 0.004])]
    P = m.coords[m.cells]
    W = np.stack([_tri_avg_quadratic(P, c) for c in coefs], axis=1)
    grad = np.zeros((m.n_cells, 4, 2))
    for q, c in enumerate(coefs):
        grad[:, q, 0] = c[1] + 2 * c[3] * C[:, 0] + c[4] * C[:, 1]
        grad[:, q, 1] = c[2] + c[4] * C[:, 0] + 2 * c[5] * C[:, 1]
    o.set_state(W, grad)
    cells = _cells_without(o.face_geometry(0), m.n_cells, None)
    rng = np.random.default_rng(1)
    for i in rng.choice(cells, 20, replace=False):
        b0, _, _, _ = o.recon_indicators(int(i))
        for q, c in enumerate(coefs):
            qx = _square_linear(c[1], 2 * c[3], c[4])      # (d q / dx)^2
            qy = _square_linear(c[2], c[4], 2 * c[5])      # (d q / dy)^2
            first = V[i] * _tri_avg_quadratic(P[i:i + 1], qx + qy)[0]
            second = V[i] ** 2 * ((2 * c[3]) ** 2 + c[4] ** 2 + (2 * c[5]) ** 2)
            np.testing.assert_allclose(b0[q], first + second, rtol=1e-9)
