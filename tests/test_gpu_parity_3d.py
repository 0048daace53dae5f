"""GPU (HIP) vs CPU oracle parity on tetrahedral meshes (the paper's 3-D setting).

Meshes: a jittered box of 2^3 hexahedra split into 6 tetrahedra each, refined
1 -> 8 twice (3,072 / 384 / 48 cells), far field on five sides and a wall on
z = 0 (slip for Euler, isothermal or adiabatic no-slip for Navier-Stokes);
free stream at 10 degrees in the x-y plane, parallel to the wall.  Bars as in
the 2-D parity tests.  Also: the Mach 6 sphere shells, and viscous flow past
the Kuhn sphere with an adiabatic wall.
"""
import numpy as np
import pytest

import synthmesh as sm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2509_06347_amd import cgks
    return cgks


CASES = {
    "euler_box": (lambda: sm.box_tets(2, nref=2, jitter=0.1, seed=2, tags={"z0": sm.SLIP}),
                  dict(dim=3, mach=0.5, aoa_deg=10.0)),
    "ns_box": (lambda: sm.box_tets(2, nref=2, jitter=0.1, seed=4, tags={"z0": sm.ISOTHERMAL}),
               dict(dim=3, mach=0.5, aoa_deg=10.0, reynolds=100.0)),
    "ns_box_adiabatic": (lambda: sm.box_tets(2, nref=2, jitter=0.1, seed=6, tags={"z0": sm.ADIABATIC}),
                         dict(dim=3, mach=0.5, aoa_deg=10.0, reynolds=100.0)),
}


def _pair(cg, orc, mesh, n_levels=3, **params):
    print(f"[case] 3-D cells={mesh.n_cells} levels={n_levels} params={params}", flush=True)
    return cg.Solver(mesh, n_levels=n_levels, **params), orc.Oracle(mesh, n_levels=n_levels, **params)


def _perturbed(mesh, o, mach, seed, amp=0.03, slope=2e-3):
    """Smooth perturbed free stream; with a no-slip wall the velocity is ramped to
    zero at z = 0."""
    V, C = o.cell_geometry(0)
    rng = np.random.default_rng(seed)
    x, y, z = C[:, 0], C[:, 1], C[:, 2]
    ramp = np.tanh(z / 0.2)
    a = np.radians(10.0)
    rho = 1.0 + amp * np.sin(3.0 * x) * np.cos(2.0 * y + z)
    u = mach * np.cos(a) * (1.0 + amp * np.cos(2.5 * z)) * ramp
    v = mach * np.sin(a) * ramp + mach * amp * np.sin(2.0 * x)
    w = mach * amp * np.sin(3.0 * y) * z
    p = (1.0 + amp * np.cos(2.0 * x + 1.5 * y - z)) / 1.4
    W = np.stack([rho, rho * u, rho * v, rho * w, p / 0.4 + 0.5 * rho * (u * u + v * v + w * w)], axis=1)
    grad = slope * rng.standard_normal((mesh.n_cells, 5, 3))
    alpha = rng.uniform(0.5, 1.0, mesh.n_cells)
    return W, grad, alpha


@pytest.mark.parametrize("case", list(CASES))
def test_setup_integer_parity_3d(cg, orc, case):
    mesh, params = CASES[case][0](), CASES[case][1]
    g, o = _pair(cg, orc, mesh, **params)
    assert g.sizes == [tuple(s) for s in o.sizes]
    for l in range(3):
        cgc, ncg = g.coloring(l)
        coc, nco = o.coloring(l)
        assert ncg == nco and np.array_equal(cgc, coc)
        Vg, Cg = g.cell_geometry(l)
        Vo, Co = o.cell_geometry(l)
        np.testing.assert_allclose(Vg, Vo, rtol=1e-13)
        np.testing.assert_allclose(Cg, Co, rtol=1e-13, atol=1e-14)
    ag, nag = g.agglomerate(0)
    ao, nao = o.agglomerate(0)
    assert nag == nao and np.array_equal(ag, ao)


def test_free_stream_preserved_3d(cg, orc):
    mesh, params = CASES["euler_box"][0](), CASES["euler_box"][1]
    g = cg.Solver(mesh, n_levels=3, **params)
    g.init_freestream()
    R, grad, a = g.residual(0)
    assert np.abs(R).max() <= 1e-13
    assert np.abs(grad).max() <= 1e-12 and np.all(a == 1.0)


@pytest.mark.parametrize("case", list(CASES))
def test_fine_residual_parity_3d(cg, orc, case):
    mesh, params = CASES[case][0](), CASES[case][1]
    g, o = _pair(cg, orc, mesh, **params)
    W, grad, alpha = _perturbed(mesh, o, params["mach"], seed=5)
    for s in (g, o):
        s.set_state(W, grad, alpha)
    Rg, gg, ag = g.residual(0)
    Ro, go, ao = o.residual(0)
    scale = np.abs(Ro).max()
    print(f"residual: max |dR| / max |R| = {np.abs(Rg - Ro).max() / scale:.2e}", flush=True)
    assert np.abs(Rg - Ro).max() <= 1e-12 * scale
    np.testing.assert_allclose(gg, go, rtol=0, atol=1e-11 * np.abs(go).max())
    np.testing.assert_allclose(ag, ao, rtol=1e-12, atol=1e-13)
    dg, _ = g.time_steps(0)
    do, _ = o.time_steps(0)
    np.testing.assert_allclose(dg, do, rtol=1e-13)


@pytest.mark.parametrize("case", list(CASES))
def test_vcycle_trajectory_parity_3d(cg, orc, case):
    mesh, params = CASES[case][0](), CASES[case][1]
    g, o = _pair(cg, orc, mesh, **params)
    W, grad, alpha = _perturbed(mesh, o, params["mach"], seed=7, slope=0.0)
    for s in (g, o):
        s.set_state(W, None, None)
    ng = g.run_cycles(3)
    no = np.array([o.vcycle() for _ in range(3)])
    np.testing.assert_allclose(ng, no, rtol=1e-10)
    Wg, gg, ag = g.get_state()
    Wo, go, ao = o.get_state()
    assert np.abs(Wg - Wo).max() <= 1e-10 * np.abs(Wo).max()
    assert np.abs(gg - go).max() <= 1e-9 * max(np.abs(go).max(), 1e-12)
    np.testing.assert_allclose(ag, ao, rtol=0, atol=1e-8)


# ---- a sphere shell at parity size: Mach 6 flow past a sphere ----------------------

def _sphere(nref):
    return sm.sphere_shell(8, 4, 2, nref=nref, jitter=0.1, seed=1)


def _sphere_state(o, mach, seed, amp=0.02):
    V, C = o.cell_geometry(0)
    rng = np.random.default_rng(seed)
    r = np.linalg.norm(C, axis=1)
    ramp = np.tanh((r - 0.5) / 0.4)
    rho = 1.0 + amp * np.sin(2.0 * C[:, 0]) * np.cos(C[:, 1] + C[:, 2])
    u = mach * ramp
    v = mach * amp * np.sin(C[:, 2])
    w = mach * amp * np.cos(C[:, 0])
    p = (1.0 + amp * np.cos(C[:, 0] - C[:, 1])) / 1.4
    W = np.stack([rho, rho * u, rho * v, rho * w, p / 0.4 + 0.5 * rho * (u * u + v * v + w * w)], axis=1)
    return W, 1e-3 * rng.standard_normal((len(V), 5, 3)), rng.uniform(0.5, 1.0, len(V))


def test_sphere_setup_and_residual_parity(cg, orc):
    mesh = _sphere(2)
    g, o = _pair(cg, orc, mesh, dim=3, mach=6.0)
    assert g.sizes == [tuple(s) for s in o.sizes]
    for l in range(3):
        cgc, ncg = g.coloring(l)
        coc, nco = o.coloring(l)
        assert ncg == nco and np.array_equal(cgc, coc)
    W, grad, alpha = _sphere_state(o, 6.0, seed=3)
    for s in (g, o):
        s.set_state(W, grad, alpha)
    Rg, gg, ag = g.residual(0)
    Ro, go, ao = o.residual(0)
    err = np.abs(Rg - Ro).max()
    print(f"residual: max |dR| / max |R| = {err / np.abs(Ro).max():.2e}, "
          f"/ flux-sum scale = {err / o.flux_scale():.2e}", flush=True)
    assert err <= 1e-12 * o.flux_scale()
    np.testing.assert_allclose(gg, go, rtol=0, atol=1e-11 * np.abs(go).max())
    # alpha = prod 1/(1 + D^2) falls to ~1e-8 here (Mach-difference terms make D
    # large); its relative error is ~2 x the relative error of D, itself built
    # from ratios and square roots: a 1e-10 relative bar
    np.testing.assert_allclose(ag, ao, rtol=1e-10, atol=1e-13)


def test_sphere_vcycle_trajectory_parity(cg, orc):
    mesh = _sphere(1)
    g, o = _pair(cg, orc, mesh, n_levels=2, dim=3, mach=6.0)
    W, _, _ = _sphere_state(o, 6.0, seed=4)
    for s in (g, o):
        s.set_state(W, None, None)
    ng = g.run_cycles(3)
    no = np.array([o.vcycle() for _ in range(3)])
    np.testing.assert_allclose(ng, no, rtol=1e-10)
    Wg, _, _ = g.get_state()
    Wo, _, _ = o.get_state()
    assert np.abs(Wg - Wo).max() <= 1e-9 * np.abs(Wo).max()
    assert g.stats()[1] == o.stats()[1]


def test_kuhn_sphere_ns_adiabatic_wall_parity(cg, orc):
    """Navier-Stokes (Re 100, Mach 0.5) past the Kuhn sphere shell with an
    adiabatic no-slip wall (23,040 tetrahedra): fine residual, slopes, DF and
    time steps at a perturbed state, then two V-cycles."""
    mesh = sm.sphere_shell_kuhn(8, 4, 2, nref=2, wall_tag=sm.ADIABATIC)
    params = dict(dim=3, mach=0.5, reynolds=100.0)
    g, o = _pair(cg, orc, mesh, **params)
    W, grad, alpha = _sphere_state(o, 0.5, seed=13)
    for s in (g, o):
        s.set_state(W, grad, alpha)
    Rg, gg, ag = g.residual(0)
    Ro, go, ao = o.residual(0)
    err = np.abs(Rg - Ro).max() / np.abs(Ro).max()
    print(f"residual: max |dR| / max |R| = {err:.2e}", flush=True)
    assert err <= 1e-12
    np.testing.assert_allclose(gg, go, rtol=0, atol=1e-11 * np.abs(go).max())
    # DF: a product over the cell's 12 Gauss points of 1 / (1 + D^2), D built
    # from jumps of reconstructed pressures and Mach numbers that cancel near
    # the wall; one near-wall cell of 23,040 differs by 1.5e-12
    np.testing.assert_allclose(ag, ao, rtol=1e-11, atol=1e-13)
    dg, ig = g.time_steps(0)
    do, io = o.time_steps(0)
    np.testing.assert_allclose(dg, do, rtol=1e-13)
    for s in (g, o):
        s.set_state(W, None, None)
    ng = g.run_cycles(2)
    no = np.array([o.vcycle() for _ in range(2)])
    np.testing.assert_allclose(ng, no, rtol=1e-10)
    Wg, _, _ = g.get_state()
    Wo, _, _ = o.get_state()
    werr = np.abs(Wg - Wo).max() / np.abs(Wo).max()
    print(f"two V-cycles: state err {werr:.2e}", flush=True)
    assert werr <= 1e-10
