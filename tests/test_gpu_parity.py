"""Parity of the HIP library (through its C ABI) against the CPU oracle.

Tolerances (the oracle is the reference):
  * colouring and agglomeration indices: bit-exact;
  * fine residual: max |R_gpu - R_orc| <= 1e-12 * max |R_orc| (stricter than
    1e-12 of the flux-sum scale max_i sum_f |S_f F_f|, which the residual
    cancels from near convergence); slopes and DF: 1e-11 relative to their
    own scale;
  * coarse residual, LU-SGS and transfers: 1e-12 relative;
  * V-cycle trajectories: per-cycle norms 1e-10 relative; state after 10
    cycles 1e-10 relative (subsonic Euler) or 1e-8 relative (Mach 8
    Navier-Stokes transient: the forming bow shock, the positivity guard and
    WENO weights whose smoothness indicators sit near epsilon amplify the
    last-bit differences of exp/erfc and FMA contraction between the CPU and
    the GPU).
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


def _pair(cg, orc, mesh, n_levels=3, use_parents=True, **params):
    print(f"[case] cells={mesh.n_cells} levels={n_levels} parents={use_parents} params={params}", flush=True)
    return (cg.Solver(mesh, n_levels=n_levels, use_parents=use_parents, **params),
            orc.Oracle(mesh, n_levels=n_levels, use_parents=use_parents, **params))


def _perturbed(mesh, o, mach, seed, amp=0.03, slope=2e-3, wall_ramp=False):
    """Smooth perturbed free stream.  With wall_ramp the velocity vanishes towards
    the cylinder wall (a no-slip profile), which keeps the interface states of a
    no-slip wall away from the near-vacuum of an impulsive hypersonic start."""
    V, C = o.cell_geometry(0)
    rng = np.random.default_rng(seed)
    x, y = C[:, 0], C[:, 1]
    ramp = np.tanh((np.hypot(x, y) - 0.5) / 0.3) if wall_ramp else 1.0
    rho = 1.0 + amp * np.sin(0.8 * x) * np.cos(0.6 * y)
    u = mach * (1.0 + amp * np.cos(0.5 * y)) * ramp
    v = mach * amp * np.sin(0.7 * x) * ramp
    p = (1.0 + amp * np.cos(0.4 * x + 0.3 * y)) / 1.4
    W = np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)], axis=1)
    grad = slope * rng.standard_normal((mesh.n_cells, 4, 2))
    alpha = rng.uniform(0.5, 1.0, mesh.n_cells)
    return W, grad, alpha


CASES = {
    "euler_small": (lambda: sm.cylinder_euler_small(), dict(mach=0.38)),
    "ns_mach8_small": (lambda: sm.annulus(32, 8, jitter=0.1, seed=1, nref=2, wall_tag=sm.ISOTHERMAL),
                       dict(mach=8.0, reynolds=1e4)),
    "ragged_farfield": (lambda: sm.annulus(13, 5, jitter=0.2, seed=3, nref=2, wall_tag=sm.FARFIELD),
                        dict(mach=0.7, aoa_deg=12.0)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_setup_integer_parity(cg, orc, case):
    mesh, params = CASES[case][0](), CASES[case][1]
    g, o = _pair(cg, orc, mesh, **params)
    assert g.sizes == [tuple(s) for s in o.sizes]
    for l in range(3):
        cgc, ncg = g.coloring(l)
        coc, nco = o.coloring(l)
        assert ncg == nco and np.array_equal(cgc, coc)
        Vg, Cg = g.cell_geometry(l)
        Vo, Co = o.cell_geometry(l)
        np.testing.assert_allclose(Vg, Vo, rtol=1e-14)
        np.testing.assert_allclose(Cg, Co, rtol=1e-13, atol=1e-14)
    ag, nag = g.agglomerate(0)
    ao, nao = o.agglomerate(0)
    assert nag == nao and np.array_equal(ag, ao)


@pytest.mark.parametrize("case", list(CASES))
def test_fine_residual_parity(cg, orc, case):
    mesh, params = CASES[case][0](), CASES[case][1]
    g, o = _pair(cg, orc, mesh, **params)
    W, grad, alpha = _perturbed(mesh, o, params["mach"], seed=5, wall_ramp="reynolds" in params)
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


def _coarse_chain(g, o, W, grad, alpha):
    """Fine step, restriction, coarse residuals and LU-SGS on levels 1 and 2,
    prolongations: every intermediate state against the oracle."""
    for s in (g, o):
        s.set_state(W, grad, alpha)
        s.smooth(0, 1)
        s.restrict(0)
    for l in (1, 2):
        Sg = g.get_level_state(l)
        So = o.get_level_state(l)
        for a, b, name in zip(Sg, So, ("W", "W0", "F", "alpha")):
            sc = max(np.abs(b).max(), 1e-300)
            assert np.abs(a - b).max() <= 1e-11 * sc, (l, name, np.abs(a - b).max() / sc)
        Rg, _, _ = g.residual(l)
        Ro, _, _ = o.residual(l)
        assert np.abs(Rg - Ro).max() <= 1e-11 * np.abs(Ro).max()
        for s in (g, o):
            s.smooth(l, 2)
        Wg = g.get_level_state(l)[0]
        Wo = o.get_level_state(l)[0]
        assert np.abs(Wg - Wo).max() <= 1e-11 * np.abs(Wo).max()
        if l == 1:
            for s in (g, o):
                s.restrict(1)
    for l in (1, 0):
        for s in (g, o):
            s.prolong(l)
    Wg, _, _ = g.get_state()
    Wo, _, _ = o.get_state()
    assert np.abs(Wg - Wo).max() <= 1e-11 * np.abs(Wo).max()


@pytest.mark.parametrize("case", list(CASES))
def test_coarse_levels_parity(cg, orc, case):
    mesh, params = CASES[case][0](), CASES[case][1]
    g, o = _pair(cg, orc, mesh, **params)
    W, grad, alpha = _perturbed(mesh, o, params["mach"], seed=6, wall_ramp="reynolds" in params)
    _coarse_chain(g, o, W, grad, alpha)


@pytest.mark.parametrize("case", ["euler_small", "ns_mach8_small"])
def test_vcycle_trajectory_parity(cg, orc, case):
    mesh, params = CASES[case][0](), CASES[case][1]
    g, o = _pair(cg, orc, mesh, **params)
    if "reynolds" in params:
        # a no-slip start: the impulsive hypersonic start is ill-conditioned at the rear wall
        W, _, _ = _perturbed(mesh, o, params["mach"], seed=7, amp=0.0, wall_ramp=True)
        g.set_state(W)
        o.set_state(W)
    else:
        g.init_freestream()
        o.init_freestream()
    ng = g.run_cycles(10)
    no = np.array([o.vcycle() for _ in range(10)])
    np.testing.assert_allclose(ng, no, rtol=1e-10)
    Wg, gg, ag = g.get_state()
    Wo, go, ao = o.get_state()
    print(f"10 cycles: state {np.abs(Wg - Wo).max() / np.abs(Wo).max():.2e}, "
          f"slopes {np.abs(gg - go).max() / max(np.abs(go).max(), 1e-12):.2e}, DF {np.abs(ag - ao).max():.2e}",
          flush=True)
    tol = 1e-8 if "reynolds" in params else 1e-10
    assert np.abs(Wg - Wo).max() <= tol * np.abs(Wo).max()
    assert np.abs(gg - go).max() <= 10 * tol * max(np.abs(go).max(), 1e-12)
    # alpha = 1 / (1 + D^2) lies in (0, 1] and D sums jumps normalised by local
    # values, so alpha is held to an absolute bar, a decade above the state's.
    np.testing.assert_allclose(ag, ao, rtol=0, atol=100 * tol)


@pytest.mark.parametrize("kappa", [0.5, 0.0])
def test_update_limit_parity(cg, orc, kappa):
    """Coarse LU-SGS under a forcing large enough to engage the update safeguard,
    then a prolongation of the resulting correction: same fractions as the oracle."""
    mesh = sm.annulus(12, 4, jitter=0.15, seed=11, nref=2, wall_tag=sm.SLIP)
    g, o = _pair(cg, orc, mesh, mach=0.5, update_limit=kappa)
    W, grad, alpha = _perturbed(mesh, o, 0.5, seed=8)
    for s in (g, o):
        s.set_state(W, grad, alpha)
        s.smooth(0, 1)
        s.restrict(0)
    V1, _ = o.cell_geometry(1)
    F = o.get_level_state(1)[2].copy()
    F[:, 0] -= 30.0 * V1
    for s in (g, o):
        s.set_level_state(1, F=F)
        s.smooth(1, 2)
    Wg, Wo = g.get_level_state(1)[0], o.get_level_state(1)[0]
    assert np.abs(Wg - Wo).max() <= 1e-11 * np.abs(Wo).max()
    sk = []
    for s in (g, o):
        s.prolong(0)
        sk.append(s.stats()[1])
    Wg, _, _ = g.get_state()
    Wo, _, _ = o.get_state()
    assert np.abs(Wg - Wo).max() <= 1e-11 * np.abs(Wo).max()
    assert sk[0] == sk[1]


AGG_CASES = {
    "2d_ragged_farfield": (lambda: sm.annulus(13, 5, jitter=0.2, seed=3, nref=2, wall_tag=sm.FARFIELD),
                           dict(mach=0.7, aoa_deg=12.0)),
    "3d_box_slip": (lambda: sm.box_tets(2, nref=2, jitter=0.1, seed=2, tags={"z0": sm.SLIP}),
                    dict(dim=3, mach=0.5, aoa_deg=10.0)),
    # meshes generated directly at the fine size (no refinement, so no nesting
    # at all): the whole hierarchy comes from Alg. 3
    "2d_unrefined_slip": (lambda: sm.annulus(48, 16, jitter=0.25, seed=7, nref=0, wall_tag=sm.SLIP),
                          dict(mach=0.4)),
    "3d_unrefined_ns_adiabatic": (lambda: sm.box_tets(5, nref=0, jitter=0.2, seed=9, tags={"z0": sm.ADIABATIC}),
                                  dict(dim=3, mach=0.5, reynolds=100.0)),
}


@pytest.mark.parametrize("case", list(AGG_CASES))
def test_agglomerated_hierarchy_parity(cg, orc, case):
    """Coarse levels built by Alg. 3 agglomeration instead of refinement parents:
    irregular agglomerates with up to 6 (2-D) or 10 (3-D) faces, the latter
    beyond the slot-parallel kernels' 8 slots (the per-cell kernels run).
    Set-up bit-exact, the coarse chain and a 3-cycle trajectory to the bars above."""
    mesh, params = AGG_CASES[case][0](), AGG_CASES[case][1]
    g, o = _pair(cg, orc, mesh, use_parents=False, **params)
    assert g.sizes == [tuple(x) for x in o.sizes]
    assert g.sizes[1][0] < mesh.n_cells and g.sizes[2][0] < g.sizes[1][0]
    for l in range(3):
        cgc, ncg = g.coloring(l)
        coc, nco = o.coloring(l)
        assert ncg == nco and np.array_equal(cgc, coc)
        Vg, Cg = g.cell_geometry(l)
        Vo, Co = o.cell_geometry(l)
        np.testing.assert_allclose(Vg, Vo, rtol=1e-13)
        np.testing.assert_allclose(Cg, Co, rtol=1e-13, atol=1e-14)
    V, C = o.cell_geometry(0)
    rng = np.random.default_rng(12)
    m, dim = params["mach"], params.get("dim", 2)
    rho = 1.0 + 0.03 * np.sin(2.0 * C[:, 0]) * np.cos(1.5 * C[:, 1])
    U = np.zeros((mesh.n_cells, dim))
    U[:, 0] = m * (1.0 + 0.03 * np.cos(C[:, 1]))
    U[:, 1] = 0.03 * m * np.sin(C[:, 0])
    p = (1.0 + 0.03 * np.cos(C[:, 0] - C[:, 1])) / 1.4
    W = np.column_stack([rho, rho[:, None] * U, p / 0.4 + 0.5 * rho * (U ** 2).sum(1)])
    grad = 1e-3 * rng.standard_normal((mesh.n_cells, dim + 2, dim))
    alpha = rng.uniform(0.5, 1.0, mesh.n_cells)
    _coarse_chain(g, o, W, grad, alpha)
    for s in (g, o):
        s.set_state(W, None, None)
    ng = g.run_cycles(3)
    no = np.array([o.vcycle() for _ in range(3)])
    np.testing.assert_allclose(ng, no, rtol=1e-10)
    Wg, _, _ = g.get_state()
    Wo, _, _ = o.get_state()
    assert np.abs(Wg - Wo).max() <= 1e-10 * np.abs(Wo).max()


def test_cfl_ramp_parity(cg, orc):
    """Impulsive Mach 3 start against an isothermal wall with a 4-cycle ramp of the
    implicit CFL: per-cycle norms and states track the oracle over the ramp and
    past it, and the first ramped cycle is bit for bit a fixed-CFL 2.5 cycle."""
    mesh = sm.annulus(12, 4, jitter=0.1, seed=5, nref=2, wall_tag=sm.ISOTHERMAL)
    params = dict(mach=3.0, reynolds=1000.0)
    g, o = _pair(cg, orc, mesh, cfl_ramp=4, **params)
    W, _, _ = _perturbed(mesh, o, 3.0, seed=9, wall_ramp=True)
    for s in (g, o):
        s.set_state(W)
    ng = g.run_cycles(6)
    no = np.array([o.vcycle() for _ in range(6)])
    np.testing.assert_allclose(ng, no, rtol=1e-9)
    Wg, _, _ = g.get_state()
    Wo, _, _ = o.get_state()
    assert np.abs(Wg - Wo).max() <= 1e-8 * np.abs(Wo).max()
    a = cg.Solver(mesh, n_levels=3, cfl_ramp=4, **params)
    b = cg.Solver(mesh, n_levels=3, cfl_imp=2.5, **params)
    for s in (a, b):
        s.set_state(W)
        s.run_cycles(1)
    for x, y in zip(a.get_state(), b.get_state()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("precision", [0, 1])
def test_shared_residual_parity(cg, orc, precision):
    """The V-cycle with one fine residual evaluation (shared_residual = 1): per-cycle
    norms and the state after 8 cycles against the oracle, from a perturbed
    state (FP32 coarse correction: the norms, which come first in each cycle,
    to 1e-10 for the first cycle; the state to the FP32 correction's bar)."""
    mesh, params = CASES["euler_small"][0](), CASES["euler_small"][1]
    g, o = _pair(cg, orc, mesh, shared_residual=1, precision=precision, **params)
    W, grad, alpha = _perturbed(mesh, o, params["mach"], seed=14)
    for s in (g, o):
        s.set_state(W, grad, alpha)
    ng = g.run_cycles(8)
    no = np.array([o.vcycle() for _ in range(8)])
    Wg, _, _ = g.get_state()
    Wo, _, _ = o.get_state()
    if precision == 0:
        np.testing.assert_allclose(ng, no, rtol=1e-10)
        assert np.abs(Wg - Wo).max() <= 1e-10 * np.abs(Wo).max()
    else:
        np.testing.assert_allclose(ng[0], no[0], rtol=1e-12)
        np.testing.assert_allclose(ng, no, rtol=1e-4)
        assert np.abs(Wg - Wo).max() <= 1e-5 * np.abs(Wo).max()


@pytest.mark.parametrize("df_relax", [2, 3])
def test_fixed_relaxation_parity(cg, orc, df_relax):
    """One fixed relaxation weight for every coarse cell instead of the DF
    weights (df_relax = 2), and the fixed-factor relaxation of the remark in
    Sec. 4.3 (df_relax = 3): the coarse chain and a 3-cycle trajectory."""
    mesh, params = CASES["ragged_farfield"][0](), CASES["ragged_farfield"][1]
    g, o = _pair(cg, orc, mesh, df_relax=df_relax, relax_beta=0.6, **params)
    W, grad, alpha = _perturbed(mesh, o, params["mach"], seed=13)
    _coarse_chain(g, o, W, grad, alpha)
    for s in (g, o):
        s.set_state(W, None, None)
    ng = g.run_cycles(3)
    no = np.array([o.vcycle() for _ in range(3)])
    np.testing.assert_allclose(ng, no, rtol=1e-10)
    Wg, _, _ = g.get_state()
    Wo, _, _ = o.get_state()
    assert np.abs(Wg - Wo).max() <= 1e-10 * np.abs(Wo).max()


@pytest.mark.parametrize("slope_relax", [0.3, 1.0])
def test_explicit_solver_parity(cg, orc, slope_relax):
    """The explicit CGKS solver (one level: the fine step alone, the baseline the
    multigrid is measured against) from the free stream on the steady Re 40
    cylinder: per-step norms and the state after 10 steps against the oracle,
    with the relaxed and with the paper's direct slope update."""
    mesh = sm.annulus(32, 8, jitter=0.15, seed=0, nref=2, wall_tag=sm.ISOTHERMAL)
    g, o = _pair(cg, orc, mesh, n_levels=1, mach=0.15, reynolds=40.0, slope_relax=slope_relax)
    for s in (g, o):
        s.init_freestream()
    ng = g.run_cycles(10)
    no = np.array([o.vcycle() for _ in range(10)])
    np.testing.assert_allclose(ng, no, rtol=1e-10)
    Wg, gg, _ = g.get_state()
    Wo, go, _ = o.get_state()
    assert np.abs(Wg - Wo).max() <= 1e-10 * np.abs(Wo).max()
    assert np.abs(gg - go).max() <= 1e-9 * np.abs(go).max()


def test_free_stream_preserved_on_gpu(cg, orc):
    mesh = sm.annulus(13, 5, jitter=0.2, seed=3, nref=2, wall_tag=sm.FARFIELD)
    g = cg.Solver(mesh, n_levels=3, mach=0.7, aoa_deg=12.0)
    g.init_freestream()
    W0, _, _ = g.get_state()
    R, gr, a = g.residual(0)
    assert np.abs(R).max() <= 1e-14 * np.abs(W0).max()
    assert np.abs(gr).max() <= 1e-12 and (a == 1.0).all()
    g.run_cycles(3)
    W1, _, _ = g.get_state()
    assert np.abs(W1 - W0).max() <= 1e-13


def test_graph_replay_is_bitwise_reproducible(cg):
    mesh = sm.cylinder_euler_small()
    runs = []
    for _ in range(2):
        g = cg.Solver(mesh, n_levels=3, mach=0.38)
        g.init_freestream()
        h = g.run_cycles(6)
        W, _, _ = g.get_state()
        runs.append((h, W))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    # graph replay equals single-cycle calls
    g = cg.Solver(mesh, n_levels=3, mach=0.38)
    g.init_freestream()
    h1 = np.array([g.vcycle() for _ in range(6)])
    W1, _, _ = g.get_state()
    assert np.array_equal(h1, runs[0][0]) and np.array_equal(W1, runs[0][1])


def test_long_trajectory_parity_viscous_steady(cg, orc):
    """25 V-cycles of a steady viscous case (Mach 0.15, Re 40, isothermal wall)
    from free stream: per-cycle norms and the final state track the oracle.  A
    longer horizon than the 10-cycle tests, so that a kernel defect that only
    shows after many cycles cannot hide."""
    mesh = sm.annulus(32, 8, jitter=0.15, seed=0, nref=2, wall_tag=sm.ISOTHERMAL)
    g, o = _pair(cg, orc, mesh, mach=0.15, reynolds=40.0)
    g.init_freestream()
    o.init_freestream()
    ng = g.run_cycles(25)
    no = np.array([o.vcycle() for _ in range(25)])
    np.testing.assert_allclose(ng, no, rtol=1e-9)
    Wg, _, _ = g.get_state()
    Wo, _, _ = o.get_state()
    assert np.abs(Wg - Wo).max() <= 1e-9 * np.abs(Wo).max()


@pytest.mark.parametrize("precision,cfl_ramp", [(0, 0), (1, 0), (1, 4)])
def test_batch_equals_individual_solves(cg, precision, cfl_ramp):
    """A batch advances each problem exactly as its own context would: fine states
    bitwise equal after 5 cycles (same kernels, per-problem parameters), norms
    equal to rounding (the batch reduces per problem in another fixed order);
    with the FP64 or the FP32 coarse correction, and with the CFL ramp (the batch
    counts its cycles from its creation, each context from its initial state)."""
    specs = [(sm.annulus(12, 4, jitter=0.1, seed=1, nref=2, wall_tag=sm.ISOTHERMAL), dict(mach=2.0, reynolds=500.0)),
             (sm.annulus(16, 4, jitter=0.2, seed=2, nref=2, wall_tag=sm.ISOTHERMAL), dict(mach=0.5, reynolds=2000.0)),
             (sm.annulus(8, 3, jitter=0.1, seed=3, nref=2, wall_tag=sm.ISOTHERMAL), dict(mach=4.0, reynolds=1e4,
                                                                                       wall_T_ratio=2.0))]
    singles, members = [], []
    for mesh, p in specs:
        for lst in (singles, members):
            s = cg.Solver(mesh, n_levels=3, precision=precision, cfl_ramp=cfl_ramp, **p)
            s.init_freestream()
            lst.append(s)
    ref = [s.run_cycles(5) for s in singles]
    batch = cg.Batch(members)
    hist = batch.run_cycles(5)
    batch.sync_states()
    for b in range(len(specs)):
        np.testing.assert_allclose(hist[b], ref[b], rtol=1e-12)
        Wb, gb, ab = members[b].get_state()
        Ws, gs, as_ = singles[b].get_state()
        assert np.array_equal(Wb, Ws) and np.array_equal(gb, gs) and np.array_equal(ab, as_)


def test_batch_solve_freezes_converged_members(cg):
    """A member that has converged stops cycling: its state stays the one it
    had at the end of the chunk of cycles in which it converged, while the
    others advance exactly as their own contexts would (the batch reads norms
    after chunks of 8, 16, ... cycles)."""
    steady = sm.annulus(12, 4, jitter=0.1, seed=5, nref=2, wall_tag=sm.FARFIELD)
    moving = sm.annulus(12, 4, jitter=0.1, seed=1, nref=2, wall_tag=sm.ISOTHERMAL)
    prm = [dict(mach=0.5, reynolds=100.0), dict(mach=0.3, reynolds=40.0)]
    members, singles = [], []
    for mesh, p in zip((steady, moving), prm):
        for lst in (members, singles):
            s = cg.Solver(mesh, n_levels=3, **p)
            s.init_freestream()
            lst.append(s)
    batch = cg.Batch(members)
    rc, cycles, status = batch.solve(tol=1e-10, max_cycles=20)
    batch.sync_states()
    assert status[0] == cg.OK and cycles[0] == 1        # the free stream is a steady state
    assert status[1] == cg.NOTCONV and cycles[1] == 20
    singles[0].run_cycles(8)                             # the first chunk
    singles[1].run_cycles(20)
    for b in range(2):
        Wb, gb, ab = members[b].get_state()
        Ws, gs, as_ = singles[b].get_state()
        assert np.array_equal(Wb, Ws) and np.array_equal(gb, gs) and np.array_equal(ab, as_), b


@pytest.mark.parametrize("dim", [2, 3])
def test_coarse_block_sizes_and_autotune_keep_the_arithmetic(cg, dim):
    """The coarse levels' slot-parallel kernels at 16, 32 and 64 cells per block,
    and the autotuner's choice, run the same per-cell arithmetic: V-cycles agree
    to rounding (the compiler may pair the multiply-adds of the differently
    sized instantiations differently), which the impulsive Mach 6 start
    amplifies over seven cycles to ~1e-12 of the state, inside the oracle
    trajectory bar (1e-10).  Equal shapes agree bit for bit.  The autotuner
    keeps the fine state and the statistics counters."""
    if dim == 2:
        mesh, prm = sm.annulus(32, 8, jitter=0.1, seed=1, nref=2, wall_tag=sm.ISOTHERMAL), dict(mach=3.0, reynolds=1e3)
    else:
        mesh, prm = sm.sphere_shell_kuhn(8, 4, 4, nref=2), dict(mach=6.0, cfl_ramp=10)
    runs = []
    for shape in ([64, 64], [64, 64], [16, 16], [32, 16], "auto"):
        s = cg.Solver(mesh, n_levels=3, **prm)
        s.init_freestream()
        h0 = s.run_cycles(3)
        if shape == "auto":
            W0, g0, a0 = s.get_state()
            st0 = s.stats()
            s.autotune()
            W1, g1, a1 = s.get_state()
            assert np.array_equal(W0, W1) and np.array_equal(g0, g1) and np.array_equal(a0, a1)
            assert s.stats() == st0
            assert all(v in (16, 32, 64) for v in s.coarse_shapes())
            shape = s.coarse_shapes()
        else:
            s.set_coarse_shapes(shape)
            assert s.coarse_shapes() == shape
        h = np.concatenate([h0, s.run_cycles(4)])
        runs.append((shape, h, s.get_state()[0]))
    # the same shapes: bit for bit
    assert np.array_equal(runs[0][1], runs[1][1]) and np.array_equal(runs[0][2], runs[1][2])
    for shape, h, W in runs[2:]:
        dh = np.abs(h - runs[0][1]).max() / np.abs(runs[0][1]).max()
        dW = np.abs(W - runs[0][2]).max() / np.abs(runs[0][2]).max()
        print(f"[case] dim {dim} coarse cells per block {shape}: norms {dh:.1e}, state {dW:.1e}", flush=True)
        assert dh <= 1e-12 and dW <= 1e-10
    with pytest.raises(cg.CgksError):
        s.set_coarse_shapes([48, 64])


def test_slip_wall_p1_option_parity(cg, orc):
    """The slip-wall p^1 option with tau_c1 = 0.1 (the pair with which the
    inviscid slip-wall cylinder converges): residual at a perturbed state and
    a 5-cycle trajectory from the free stream, against the oracle."""
    mesh = sm.annulus(32, 8, jitter=0.15, seed=0, nref=1, wall_tag=sm.SLIP)
    params = dict(mach=0.38, tau_c1=0.1, slip_wall_p1=1)
    g, o = _pair(cg, orc, mesh, **params)
    W, grad, alpha = _perturbed(mesh, o, 0.38, seed=21)
    for s in (g, o):
        s.set_state(W, grad, alpha)
    Rg, gg, ag = g.residual(0)
    Ro, go, ao = o.residual(0)
    err = np.abs(Rg - Ro).max() / np.abs(Ro).max()
    print(f"residual: max |dR| / max |R| = {err:.2e}", flush=True)
    assert err <= 1e-12
    np.testing.assert_allclose(gg, go, rtol=0, atol=1e-11 * np.abs(go).max())
    np.testing.assert_allclose(ag, ao, rtol=1e-12, atol=1e-13)
    for s in (g, o):
        s.init_freestream()
    ng = g.run_cycles(5)
    no = np.array([o.vcycle() for _ in range(5)])
    np.testing.assert_allclose(ng, no, rtol=1e-10)
    Wg, _, _ = g.get_state()
    Wo, _, _ = o.get_state()
    assert np.abs(Wg - Wo).max() <= 1e-10 * np.abs(Wo).max()
