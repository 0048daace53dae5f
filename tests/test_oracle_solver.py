"""Pins of the oracle's residual, smoothers and transfers (Secs. 2-5).

Checks use invariants and special cases the paper's equations fix:
free-stream preservation, discrete conservation in a closed box, exactness of
the large-stencil reconstruction for quadratics, equality of multi-colour
and sequential LU-SGS, the alpha -> 0 limits of the DF relaxation and of the
DF prolongation, and the FAS identity (coarse RHS at W0 = restricted residual).
"""
import numpy as np
import pytest

import synthmesh as sm

G = 1.4


def cons_field(rho, u, v, p):
    return np.stack([rho, rho * u, rho * v, p / (G - 1) + 0.5 * rho * (u * u + v * v)], axis=-1)


def smooth_state(C, mach=0.5, amp=0.05):
    x, y = C[:, 0], C[:, 1]
    rho = 1.0 + amp * np.sin(0.7 * x + 0.3) * np.cos(0.5 * y)
    u = mach * (1.0 + amp * np.cos(0.4 * y))
    v = mach * amp * np.sin(0.6 * x)
    p = 1.0 / G * (1.0 + amp * np.cos(0.3 * x - 0.2 * y))
    return cons_field(rho, u, v, p)


@pytest.fixture(scope="module")
def ff_mesh():
    return sm.annulus(12, 4, jitter=0.15, seed=3, nref=2, wall_tag=sm.FARFIELD)


def test_free_stream_preservation(orc, ff_mesh):
    o = orc.Oracle(ff_mesh, n_levels=3, mach=0.7, aoa_deg=10.0)
    o.init_freestream()
    W0, _, _ = o.get_state()
    R, g, a = o.residual(0)
    fg = o.face_geometry(0)
    scale = fg["S"].max() * np.abs(W0).max()
    assert np.abs(R).max() <= 1e-13 * scale
    assert np.abs(g).max() <= 1e-12
    assert (a == 1.0).all()
    o.vcycle()
    W1, _, _ = o.get_state()
    assert np.abs(W1 - W0).max() <= 1e-13


def test_closed_box_conserves_mass_and_energy(orc):
    m = sm.structured_square(5, jitter=0.2, seed=4, tag=sm.SLIP)
    for re in (0.0, 200.0):
        o = orc.Oracle(m, n_levels=1, mach=0.5, reynolds=re)
        V, C = o.cell_geometry(0)
        o.set_state(smooth_state(C))
        R, _, _ = o.residual(0)
        # interior fluxes cancel pairwise and the slip walls carry no mass or energy
        for q in (0, 3):
            assert abs(R[:, q].sum()) <= 1e-14 * np.abs(R[:, q]).sum() + 1e-16


def _tri_avg_quadratic(P, coef):
    """Exact average over triangles of c0 + c1 x + c2 y + c3 x^2 + c4 xy + c5 y^2."""
    x0, x1, x2 = P[:, 0, 0], P[:, 1, 0], P[:, 2, 0]
    y0, y1, y2 = P[:, 0, 1], P[:, 1, 1], P[:, 2, 1]
    ax, ay = (x0 + x1 + x2) / 3, (y0 + y1 + y2) / 3
    axx = (x0 * x0 + x1 * x1 + x2 * x2 + x0 * x1 + x1 * x2 + x2 * x0) / 6
    ayy = (y0 * y0 + y1 * y1 + y2 * y2 + y0 * y1 + y1 * y2 + y2 * y0) / 6
    axy = (2 * (x0 * y0 + x1 * y1 + x2 * y2) + x0 * y1 + x1 * y0 + x1 * y2 + x2 * y1 + x2 * y0 + x0 * y2) / 12
    c = coef
    return c[0] + c[1] * ax + c[2] * ay + c[3] * axx + c[4] * axy + c[5] * ayy


def test_large_stencil_reproduces_quadratics(orc):
    """p^2 matches the neighbours' averages exactly and the slopes in the LS sense,
    so a quadratic field is reproduced exactly (Sec. 3.1)."""
    m = sm.annulus(12, 4, jitter=0.15, seed=9, nref=1, wall_tag=sm.FARFIELD)
    o = orc.Oracle(m, n_levels=1, mach=0.3)
    V, C = o.cell_geometry(0)
    rng = np.random.default_rng(0)
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
    fg = o.face_geometry(0)
    interior = np.bincount(fg["LR"][fg["LR"][:, 1] >= 0].ravel(), minlength=m.n_cells)
    for i in rng.choice(np.where(interior == 3)[0], 25, replace=False):
        for x in (C[i], P[i, 0] * 0.6 + 0.4 * C[i], P[i, 2]):
            _, _, p2, _, _ = o.recon_eval(int(i), x)
            exact = np.array([c[0] + c[1] * x[0] + c[2] * x[1] + c[3] * x[0] ** 2 + c[4] * x[0] * x[1]
                              + c[5] * x[1] ** 2 for c in coefs])
            np.testing.assert_allclose(p2, exact, rtol=0, atol=1e-11)


def test_constant_data_reconstructs_constant(orc, ff_mesh):
    o = orc.Oracle(ff_mesh, n_levels=1, mach=0.4)
    o.init_freestream()
    W, _, _ = o.get_state()
    V, C = o.cell_geometry(0)
    for i in (0, 17, 100):
        Wx, gx, p2, p1, w = o.recon_eval(i, C[i] + 0.01)
        np.testing.assert_allclose(Wx, W[i], rtol=1e-14)
        assert np.abs(gx).max() <= 1e-12
        np.testing.assert_allclose(w, 0.95, rtol=1e-15)


def _prepared(orc, mesh, **kw):
    o = orc.Oracle(mesh, n_levels=3, **kw)
    V, C = o.cell_geometry(0)
    o.set_state(smooth_state(C, mach=kw.get("mach", 0.5)))
    return o


def test_multicolour_lusgs_equals_sequential_lusgs(orc, small_mesh):
    """Cells of one colour never interact, so Alg. 2 equals the classical sequential
    LU-SGS in (colour, index) order, bit for bit (Sec. 4.2)."""
    a = _prepared(orc, small_mesh, mach=0.5)
    b = _prepared(orc, small_mesh, mach=0.5)
    for o in (a, b):
        o.smooth(0, 1)
        o.restrict(0)
    a.smooth(1, 3)
    b.smooth_sequential(1, 3)
    Wa = a.get_level_state(1)[0]
    Wb = b.get_level_state(1)[0]
    assert np.array_equal(Wa, Wb)
    assert np.abs(Wa - a.get_level_state(1)[1]).max() > 0  # the sweep did something


@pytest.fixture(scope="module")
def small_mesh():
    return sm.annulus(12, 4, jitter=0.15, seed=11, nref=2, wall_tag=sm.SLIP)


def test_df_relaxation_zero_is_explicit_step(orc, small_mesh):
    """alpha -> 0 turns the relaxed LU-SGS into the explicit step dW = dt/V * RHS (Sec. 4.3 remark)."""
    o = _prepared(orc, small_mesh, mach=0.5)
    o.smooth(0, 1)
    o.restrict(0)
    W, W0, F, a = o.get_level_state(1)
    o.set_level_state(1, alpha=np.zeros_like(a))
    R, _, _ = o.residual(1)
    dte, _ = o.time_steps(1)
    V, _ = o.cell_geometry(1)
    o.smooth(1, 1)
    W1 = o.get_level_state(1)[0]
    np.testing.assert_allclose(W1 - W, (dte / V)[:, None] * (-R), rtol=1e-12, atol=1e-15)


def test_restriction_and_fas_identities(orc, small_mesh):
    o = _prepared(orc, small_mesh, mach=0.5)
    o.smooth(0, 1)
    Wf, _, _ = o.get_state()
    Rf, _, af = o.residual(0)           # residual at the smoothed state
    o.restrict(0)
    W, W0, F, a1 = o.get_level_state(1)
    V0, _ = o.cell_geometry(0)
    V1, _ = o.cell_geometry(1)
    p0 = small_mesh.parents[0]
    for q in range(4):
        assert (V1 * W0[:, q]).sum() == pytest.approx((V0 * Wf[:, q]).sum(), rel=1e-13)
    np.testing.assert_allclose(a1, [af[p0 == I].min() for I in range(len(a1))])
    # FAS: the coarse right-hand side at W0 is the restricted fine residual
    Rc, _, _ = o.residual(1)
    ref = np.stack([np.bincount(p0, weights=Rf[:, q]) for q in range(4)], axis=1)
    np.testing.assert_allclose(Rc, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_restriction_of_constant_is_exact(orc, ff_mesh):
    o = orc.Oracle(ff_mesh, n_levels=3, mach=0.6)
    o.init_freestream()
    W, _, _ = o.get_state()
    o.restrict(0)
    for l in (1, 2):
        if l == 2:
            o.restrict(1)
        _, W0, _, _ = o.get_level_state(l)
        np.testing.assert_allclose(W0, np.broadcast_to(W[0], W0.shape), rtol=1e-14)


def test_df_prolongation_zero_is_identity(orc, small_mesh):
    o = _prepared(orc, small_mesh, mach=0.5)
    o.smooth(0, 1)
    o.restrict(0)
    o.smooth(1, 2)
    W, g, a = o.get_state()
    o.set_state(W, g, np.zeros_like(a))
    o.prolong(0)
    W2, _, _ = o.get_state()
    assert np.array_equal(W, W2)
    o.set_state(W, g, np.ones_like(a))
    o.prolong(0)
    W3, _, _ = o.get_state()
    Wc, W0c, _, _ = o.get_level_state(1)
    p0 = small_mesh.parents[0]
    np.testing.assert_allclose(W3, W + (Wc - W0c)[p0], rtol=1e-14, atol=1e-15)


def test_vcycle_is_stable_on_agglomerated_levels(orc):
    m = sm.annulus(12, 4, jitter=0.1, seed=2, nref=2, wall_tag=sm.SLIP)
    o = orc.Oracle(m, n_levels=3, use_parents=False, mach=0.4)
    o.init_freestream()
    norms = [o.vcycle() for _ in range(5)]
    assert all(np.isfinite(norms)) and norms[-1] < norms[0]


def _rho_e(W):
    return W[:, 3] - 0.5 * (W[:, 1] ** 2 + W[:, 2] ** 2) / W[:, 0]


@pytest.mark.parametrize("kappa,drho,theta", [
    (0.5, -0.3, 1.0),     # rho 0.7 >= 0.5: whole correction
    (0.5, -0.8, 0.5),     # rho 0.2 < 0.5, half -> 0.6
    (0.5, -1.5, 0.25),    # 1 and 1/2 fail, a quarter -> 0.625
    (0.0, -0.8, 1.0),     # kappa 0: whole while rho, p stay positive
    (0.0, -1.2, 0.0),     # kappa 0: skipped when rho would be negative
])
def test_prolongation_update_limit_closed_form(orc, ff_mesh, kappa, drho, theta):
    """The update safeguard on the injected correction, against hand-computed
    fractions: with momentum and energy unchanged, rho e also stays above half."""
    o = orc.Oracle(ff_mesh, n_levels=2, mach=0.5, df_prolong=0, update_limit=kappa)
    o.init_freestream()
    W, _, _ = o.get_state()
    _, W0c, _, _ = o.get_level_state(1)
    Wc = W0c.copy()
    Wc[:, 0] = W0c[:, 0] + drho
    o.set_level_state(1, W=Wc, W0=W0c)
    skips0 = o.stats()[1]
    o.prolong(0)
    W2, _, _ = o.get_state()
    d = (W0c[0, 0] + drho) - W0c[0, 0]          # the correction as the oracle forms it
    expect = W.copy()
    expect[:, 0] = W[:, 0] + theta * d
    assert np.array_equal(W2, expect)
    assert o.stats()[1] - skips0 == (0 if theta == 1.0 else len(W))


@pytest.mark.parametrize("scale", [1.0, 30.0, 1e3])
def test_lusgs_update_limit_bounds_the_drop(orc, small_mesh, scale):
    """A large mass-sink forcing on level 1: no cell loses more than kappa = 1/2
    of its rho or rho e in one LU-SGS iteration, and the level still moves."""
    o = _prepared(orc, small_mesh, mach=0.5, update_limit=0.5)
    o.smooth(0, 1)
    o.restrict(0)
    W, W0, F, a = o.get_level_state(1)
    V1, _ = o.cell_geometry(1)
    F2 = F.copy()
    F2[:, 0] -= scale * V1
    o.set_level_state(1, F=F2)
    o.smooth(1, 1)
    W1 = o.get_level_state(1)[0]
    assert np.all(W1[:, 0] >= 0.5 * W[:, 0])
    assert np.all(_rho_e(W1) >= 0.5 * _rho_e(W))
    assert np.abs(W1 - W).max() > 0


# ---- 3-D (tetrahedra) ------------------------------------------------------

def test_shared_residual_cycle_is_a_composition_of_pinned_steps(orc, small_mesh):
    """shared_residual = 1: the V-cycle restricts W^n with its own residual, solves
    the coarse levels, takes the fine step from W^n and prolongs onto its
    result.  Bit for bit: restrict(0) at W^n, 6 LU-SGS iterations, restrict(1),
    6 iterations, prolong(1), then (W^n, slopes and DF of W^n restored: restrict
    stores the new DF, which the reconstruction uses) one fine step and
    prolong(0), each pinned above."""
    A = _prepared(orc, small_mesh, mach=0.5, shared_residual=1)
    B = _prepared(orc, small_mesh, mach=0.5)
    C = _prepared(orc, small_mesh, mach=0.5)
    A.smooth(0, 1)                    # a state with slopes and DF values
    S = A.get_state()
    for o in (A, B, C):
        o.set_state(*S)
    A.vcycle()
    B.restrict(0)
    B.smooth(1, 6)
    B.restrict(1)
    B.smooth(2, 6)
    B.prolong(1)
    B.set_state(*S)
    B.smooth(0, 1)
    B.prolong(0)
    for x, y in zip(A.get_state(), B.get_state()):
        assert np.array_equal(x, y)
    C.vcycle()                        # the paper's cycle restricts the smoothed state
    assert not np.array_equal(C.get_state()[0], A.get_state()[0])


def test_fixed_relaxation_reduces_to_pinned_cases(orc, small_mesh):
    """df_relax = 2 (one relaxation weight beta for every coarse cell): beta = 1 is
    the fully implicit LU-SGS bit for bit, and a fixed beta is the DF relaxation
    with alpha = beta in every cell (whose alpha -> 0 limit is pinned above)."""
    def coarse(**kw):
        o = _prepared(orc, small_mesh, mach=0.5, **kw)
        o.smooth(0, 1)
        o.restrict(0)
        return o
    a, b = coarse(df_relax=2, relax_beta=1.0), coarse(df_relax=0)
    for o in (a, b):
        o.smooth(1, 2)
    Wa, Wb = a.get_level_state(1)[0], b.get_level_state(1)[0]
    assert np.array_equal(Wa, Wb)
    c, d = coarse(df_relax=2, relax_beta=0.6), coarse(df_relax=1)
    n1 = d.get_level_state(1)[3].shape[0]
    d.set_level_state(1, alpha=np.full(n1, 0.6))
    for o in (c, d):
        o.smooth(1, 2)
    Wc, Wd = c.get_level_state(1)[0], d.get_level_state(1)[0]
    assert np.array_equal(Wc, Wd)
    assert not np.array_equal(Wc, Wa)


def test_fixed_factor_relaxation_reduces_to_pinned_cases(orc, small_mesh):
    """df_relax = 3 (the fixed-factor relaxation of the remark in Sec. 4.3,
    beta on the implicit time term and (1 - beta) V/dt_i times the previous
    increment on the right-hand side): beta = 1 is the fully implicit LU-SGS bit
    for bit; the first iteration after restriction (no previous increment) is
    the fully implicit iteration at the implicit CFL divided by beta (bit for
    bit for beta = 1/2, an exact scaling); the second iteration is not (the
    previous increment enters)."""
    def coarse(**kw):
        o = _prepared(orc, small_mesh, mach=0.5, **kw)
        o.smooth(0, 1)
        o.restrict(0)
        return o
    a, b = coarse(df_relax=3, relax_beta=1.0), coarse(df_relax=0)
    for o in (a, b):
        o.smooth(1, 2)
    assert np.array_equal(a.get_level_state(1)[0], b.get_level_state(1)[0])
    c, d = coarse(df_relax=3, relax_beta=0.5), coarse(df_relax=0, cfl_imp=20.0)
    for o in (c, d):
        o.smooth(1, 1)
    Wc, Wd = c.get_level_state(1)[0], d.get_level_state(1)[0]
    assert np.array_equal(Wc, Wd)
    for o in (c, d):
        o.smooth(1, 1)
    Wc2, Wd2 = c.get_level_state(1)[0], d.get_level_state(1)[0]
    assert not np.array_equal(Wc2, Wd2)
    # the previous increment is cleared by the next restriction
    e = coarse(df_relax=3, relax_beta=0.5)
    e.smooth(1, 3)
    e.restrict(0)
    f = coarse(df_relax=0, cfl_imp=20.0)
    f.restrict(0)
    for o in (e, f):
        o.smooth(1, 1)
    assert np.array_equal(e.get_level_state(1)[0], f.get_level_state(1)[0])


def test_cfl_ramp_cycles_equal_fixed_cfl_cycles(orc, small_mesh):
    """The start-up ramp of N cycles runs the k-th V-cycle after a state is set at
    CFL cfl_imp * k / N: with N = 4 and cfl_imp = 10 the first two cycles are,
    bit for bit, fixed-CFL cycles at 2.5 and 5 (each scaling exact in binary),
    every cycle from the fourth on is a plain cfl_imp cycle, and setting a state
    restarts the count."""
    kw = dict(mach=0.5, cfl_imp=10.0)
    ramp = _prepared(orc, small_mesh, cfl_ramp=4, **kw)
    start = ramp.get_state()
    states = []
    for _ in range(5):
        ramp.vcycle()
        states.append(ramp.get_state())
    for k, cfl in ((0, 2.5), (1, 5.0), (3, 10.0), (4, 10.0)):
        fixed = orc.Oracle(small_mesh, n_levels=3, mach=0.5, cfl_imp=cfl)
        fixed.set_state(*(start if k == 0 else states[k - 1]))
        fixed.vcycle()
        for a, b in zip(fixed.get_state(), states[k]):
            assert np.array_equal(a, b), (k, cfl)
    # the third cycle (CFL 7.5) differs from a full-CFL cycle: the ramp is live
    full = orc.Oracle(small_mesh, n_levels=3, **kw)
    full.set_state(*states[1])
    full.vcycle()
    assert not np.array_equal(full.get_state()[0], states[2][0])
    # set_state restarts the ramp: the next cycle is a CFL-2.5 cycle again
    ramp.set_state(*start)
    ramp.vcycle()
    for a, b in zip(ramp.get_state(), states[0]):
        assert np.array_equal(a, b)
    # outside a V-cycle the implicit time step follows the last cycle's CFL
    ref = orc.Oracle(small_mesh, n_levels=3, **kw)
    ramp.vcycle()
    ref.set_state(*ramp.get_state())
    np.testing.assert_array_equal(ramp.time_steps(0)[1], 0.5 * ref.time_steps(0)[1])
    np.testing.assert_array_equal(ramp.time_steps(0)[0], ref.time_steps(0)[0])


def _tet_mesh(**kw):
    return sm.box_tets(2, nref=1, jitter=0.1, seed=kw.pop("seed", 6), **kw)


def cons_field_3d(C, mach=0.5, amp=0.05):
    x, y, z = C[:, 0], C[:, 1], C[:, 2]
    rho = 1.0 + amp * np.sin(2.0 * x + 0.3) * np.cos(1.5 * y - z)
    u = mach * (1.0 + amp * np.cos(2.0 * z))
    v = mach * amp * np.sin(1.7 * x)
    w = mach * amp * np.cos(2.1 * y)
    p = 1.0 / G * (1.0 + amp * np.cos(1.3 * x - 0.7 * y + z))
    return np.stack([rho, rho * u, rho * v, rho * w, p / (G - 1) + 0.5 * rho * (u * u + v * v + w * w)], axis=-1)


def test_free_stream_preservation_3d(orc):
    m = _tet_mesh()
    o = orc.Oracle(m, n_levels=2, dim=3, mach=0.7, aoa_deg=10.0)
    o.init_freestream()
    W0, _, _ = o.get_state()
    R, g, a = o.residual(0)
    assert np.abs(R).max() <= 1e-15 and np.abs(g).max() <= 1e-12 and (a == 1.0).all()
    o.vcycle()
    assert np.abs(o.get_state()[0] - W0).max() <= 1e-13


def test_closed_box_conserves_mass_and_energy_3d(orc):
    m = _tet_mesh(tags={k: sm.SLIP for k in ("x0", "x1", "y0", "y1", "z0", "z1")})
    for re in (0.0, 200.0):
        o = orc.Oracle(m, n_levels=1, dim=3, mach=0.5, reynolds=re)
        V, C = o.cell_geometry(0)
        o.set_state(cons_field_3d(C))
        R, _, _ = o.residual(0)
        for q in (0, 4):
            assert abs(R[:, q].sum()) <= 1e-14 * np.abs(R[:, q]).sum() + 1e-16


def _tet_avg_quadratic(P, c):
    """Exact average over tetrahedra of c0 + sum_a c_a x_a + sum_{a<=b} c_ab x_a x_b:
    the mean of x_a x_b is (sum_i x_ia x_ib + (sum_i x_ia)(sum_i x_ib)) / 20."""
    s = P.sum(axis=1)
    out = c[0] + sum(c[1 + a] * s[:, a] / 4 for a in range(3))
    k = 4
    for a in range(3):
        for b in range(a, 3):
            out = out + c[k] * ((P[:, :, a] * P[:, :, b]).sum(axis=1) + s[:, a] * s[:, b]) / 20
            k += 1
    return out


def _quad3(c, x):
    v = c[0] + sum(c[1 + a] * x[a] for a in range(3))
    k = 4
    for a in range(3):
        for b in range(a, 3):
            v += c[k] * x[a] * x[b]
            k += 1
    return v


def _quad3_grad(c, x):
    g = np.array([c[1], c[2], c[3]], dtype=float)
    k = 4
    for a in range(3):
        for b in range(a, 3):
            g[a] += c[k] * x[b]
            g[b] += c[k] * x[a]
            k += 1
    return g


def test_large_stencil_reproduces_quadratics_3d(orc):
    """On tetrahedra, p^2 (9 terms) fits 4 neighbour averages exactly and 12 slope
    rows in the least-squares sense: quadratic data are reproduced exactly."""
    m = _tet_mesh(seed=8)
    o = orc.Oracle(m, n_levels=1, dim=3, mach=0.3)
    V, C = o.cell_geometry(0)
    rng = np.random.default_rng(1)
    coefs = [rng.normal(scale=[1.0] + [0.05] * 3 + [0.02] * 6) for _ in range(5)]
    coefs[0][0] = 1.0
    coefs[4][0] = 2.5
    P = m.coords[m.cells]
    W = np.stack([_tet_avg_quadratic(P, c) for c in coefs], axis=1)
    grad = np.stack([np.array([_quad3_grad(c, x) for x in C]) for c in coefs], axis=1)
    o.set_state(W, grad)
    fg = o.face_geometry(0)
    interior = np.bincount(fg["LR"][fg["LR"][:, 1] >= 0].ravel(), minlength=m.n_cells)
    for i in rng.choice(np.where(interior == 4)[0], 15, replace=False):
        for x in (C[i], P[i, 0] * 0.6 + 0.4 * C[i], P[i, 3]):
            _, _, p2, _, _ = o.recon_eval(int(i), x)
            np.testing.assert_allclose(p2, [_quad3(c, x) for c in coefs], rtol=0, atol=1e-11)


def test_multicolour_lusgs_equals_sequential_lusgs_3d(orc):
    m = sm.box_tets(2, nref=2, jitter=0.1, seed=3, tags={"z0": sm.SLIP})
    runs = []
    for seq in (False, True):
        o = orc.Oracle(m, n_levels=3, dim=3, mach=0.5)
        V, C = o.cell_geometry(0)
        o.set_state(cons_field_3d(C))
        o.smooth(0, 1)
        o.restrict(0)
        (o.smooth_sequential if seq else o.smooth)(1, 2)
        runs.append(o.get_level_state(1)[0])
    assert np.array_equal(runs[0], runs[1])


def _cells_touching(mesh, tag):
    """Indices of the cells with a boundary face of the given tag, and of their
    face neighbours (cells sharing dim nodes with one of them)."""
    nodes = set()
    faces = [tuple(sorted(f)) for f, t in zip(mesh.bfaces, mesh.btags) if t == tag]
    cells = [tuple(sorted(c)) for c in mesh.cells]
    wall = {i for i, c in enumerate(cells) for f in faces if set(f) <= set(c)}
    near = set(wall)
    wall_sets = [set(cells[i]) for i in wall]
    for i, c in enumerate(cells):
        if any(len(set(c) & w) == mesh.dim for w in wall_sets):
            near.add(i)
    return wall, near


def test_slip_wall_p1_option_acts_on_slip_wall_cells_only(orc):
    """The slip_wall_p1 option (not the paper's reconstruction) replaces the
    combined polynomial of slip-wall cells by p^1: without slip walls it
    changes nothing bit for bit; with them it changes the residual of the
    slip-wall cells and of their face neighbours (whose faces see those
    polynomials) and of no other cell."""
    ff = sm.annulus(12, 4, jitter=0.15, seed=3, nref=1, wall_tag=sm.FARFIELD)
    wall = sm.annulus(12, 4, jitter=0.15, seed=3, nref=1, wall_tag=sm.SLIP)
    res = []
    for opt in (0, 1):
        o = orc.Oracle(ff, n_levels=1, mach=0.4, slip_wall_p1=opt)
        V, C = o.cell_geometry(0)
        o.set_state(smooth_state(C, mach=0.4), None, None)
        res.append(o.residual(0))
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)
    o0 = orc.Oracle(wall, n_levels=1, mach=0.4)
    o1 = orc.Oracle(wall, n_levels=1, mach=0.4, slip_wall_p1=1)
    V, C = o0.cell_geometry(0)
    W = smooth_state(C, mach=0.4)
    for o in (o0, o1):
        o.set_state(W, None, None)
    R0, _, _ = o0.residual(0)
    R1, _, _ = o1.residual(0)
    wall_cells, near = _cells_touching(wall, sm.SLIP)
    changed = set(np.nonzero(np.any(R0 != R1, axis=1))[0].tolist())
    assert changed and changed <= near
    assert wall_cells <= changed


@pytest.mark.parametrize("dim", [2, 3])
def test_sampled_residual_equals_full_residual(orc, dim):
    """orc_residual_cells (the residual of a sample of cells, for checking meshes
    too large for the whole residual) equals the full residual's rows bit for
    bit, boundary cells included."""
    if dim == 2:
        mesh = sm.annulus(12, 4, jitter=0.15, seed=3, nref=1, wall_tag=sm.ISOTHERMAL)
        prm = dict(mach=0.5, reynolds=100.0)
    else:
        mesh = sm.sphere_shell_kuhn(4, 2, 2, nref=1)
        prm = dict(dim=3, mach=2.0)
    o = orc.Oracle(mesh, n_levels=1, **prm)
    V, C = o.cell_geometry(0)
    rng = np.random.default_rng(4)
    W, _, _ = o.get_state()
    o.init_freestream()
    W, _, _ = o.get_state()
    W = W * (1.0 + 0.02 * rng.standard_normal(W.shape[0]))[:, None]
    grad = 1e-3 * rng.standard_normal((mesh.n_cells, dim + 2, dim))
    alpha = rng.uniform(0.5, 1.0, mesh.n_cells)
    o.set_state(W, grad, alpha)
    R, g, a = o.residual(0)
    cells = np.unique(np.concatenate([rng.choice(mesh.n_cells, 40, replace=False), [0, mesh.n_cells - 1]]))
    Rs, gs, as_ = o.residual_cells(cells)
    assert np.array_equal(Rs, R[cells]) and np.array_equal(gs, g[cells]) and np.array_equal(as_, a[cells])
