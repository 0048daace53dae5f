"""Pins of the oracle's gas-kinetic pieces against independent mathematics.

Each check uses something other than the oracle's own formulas: Gauss-Hermite
or adaptive quadrature of the Maxwellian, the Chapman-Enskog closed form of
the Navier-Stokes fluxes, the Euler flux, or the exact limits tau -> 0 and
tau -> infinity of the BGK integral solution (Sec. 2.3, Eq. integral1).
"""
import math

import numpy as np
import pytest
from numpy.polynomial.hermite import hermgauss
from scipy import integrate
from scipy.special import erfc

GAMMA = 1.4


def K2(gamma=GAMMA):
    return (4.0 - 2.0 * gamma) / (gamma - 1.0)


def cons(rho, u, p, gamma=GAMMA):
    u = np.asarray(u, dtype=float)
    return np.concatenate([[rho], rho * u, [p / (gamma - 1.0) + 0.5 * rho * u @ u]])


def euler_flux(W, n, gamma=GAMMA):
    d = len(W) - 2
    rho = W[0]
    u = W[1:1 + d] / rho
    p = (gamma - 1.0) * (W[-1] - 0.5 * rho * u @ u)
    un = u @ n
    return np.concatenate([[rho * un], rho * u * un + p * np.asarray(n), [(W[-1] + p) * un]])


# ---------------------------------------------------------------- moments --

@pytest.mark.parametrize("U,lam", [(0.3, 0.7), (-1.7, 2.5), (4.0, 0.35), (0.0, 1.0)])
def test_full_range_moments_vs_gauss_hermite(orc, U, lam):
    x, w = hermgauss(60)
    u = U + x / math.sqrt(lam)
    ref = np.array([(w * u ** k).sum() / math.sqrt(math.pi) for k in range(12)])
    got = orc.moments(U, lam, 0)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("U,lam", [(0.3, 0.7), (-1.7, 2.5), (2.0, 0.35), (0.0, 1.0)])
def test_half_range_moments_vs_quadrature(orc, U, lam):
    g = lambda u, k: u ** k * math.sqrt(lam / math.pi) * math.exp(-lam * (u - U) ** 2)
    pos = orc.moments(U, lam, +1)
    neg = orc.moments(U, lam, -1)
    for k in range(9):
        rp = integrate.quad(g, 0.0, np.inf, args=(k,), epsabs=0, epsrel=1e-13, limit=200)[0]
        rn = integrate.quad(g, -np.inf, 0.0, args=(k,), epsabs=0, epsrel=1e-13, limit=200)[0]
        assert abs(pos[k] - rp) <= 1e-10 * max(1.0, abs(rp))
        assert abs(neg[k] - rn) <= 1e-10 * max(1.0, abs(rn))
    np.testing.assert_allclose(pos + neg, orc.moments(U, lam, 0), rtol=1e-13, atol=1e-13)
    assert pos[0] == pytest.approx(0.5 * erfc(-math.sqrt(lam) * U), rel=1e-15)


def _psi_quadrature(rho, U, lam, dim, K, nodes=24):
    """Tensor Gauss-Hermite quadrature of the Maxwellian in (u_1..u_d, xi_1..xi_K)."""
    x, w = hermgauss(nodes)
    xk, wk = hermgauss(6)
    grids = np.meshgrid(*([x] * dim), indexing="ij")
    wts = np.ones_like(grids[0])
    for d, gw in enumerate(np.meshgrid(*([w] * dim), indexing="ij")):
        wts = wts * gw
    vel = [U[d] + grids[d] / math.sqrt(lam) for d in range(dim)]
    # internal degrees of freedom: each xi_i ~ N(0, 1/(2 lam)); xi^2 = sum xi_i^2
    xis = np.meshgrid(*([xk] * int(K)), indexing="ij")
    wx = np.ones_like(xis[0])
    for gw in np.meshgrid(*([wk] * int(K)), indexing="ij"):
        wx = wx * gw
    xi2 = sum((g / math.sqrt(lam)) ** 2 for g in xis)
    norm = math.pi ** ((dim + int(K)) / 2.0)
    return vel, wts, xi2.ravel(), wx.ravel(), norm


def test_moment_solve_inverts_the_moment_map(orc):
    """<a psi> = b by independent quadrature (Sec. 2.3, Eq. co)."""
    rng = np.random.default_rng(3)
    for dim in (2, 3):
        K = 2.0 / (GAMMA - 1.0) - dim
        rho, U, p = 1.3, rng.uniform(-1, 1, dim), 0.8
        lam = rho / (2 * p)
        W = cons(rho, U, p)
        b = rng.normal(size=dim + 2)
        a = orc.moment_solve(W, b, dim=dim)
        vel, wts, xi2, wx, norm = _psi_quadrature(rho, U, lam, dim, K)
        e = 0.5 * (sum(v ** 2 for v in vel)[..., None] + xi2[None, :])
        psi = [np.ones_like(e)] + [np.broadcast_to(v[..., None], e.shape) for v in vel] + [e]
        s = sum(a[k] * psi[k] for k in range(dim + 2))
        W8 = wts[..., None] * wx[None, :]
        got = np.array([(W8 * s * psi[k]).sum() / norm for k in range(dim + 2)])
        np.testing.assert_allclose(got, b, rtol=1e-10, atol=1e-10)


# ---------------------------------------------------------- time integrals --

@pytest.mark.parametrize("dt,tau", [(1.0, 0.1), (0.3, 0.9), (2e-3, 1e-4), (1.0, 5.0)])
def test_time_coefficients_vs_quadrature(orc, dt, tau):
    """q-coefficients = integrals over [0,dt] of C1, C2, C3 and the kinetic weights (Eq. dis2)."""
    fns = [lambda t: 1 - math.exp(-t / tau),
           lambda t: (t + tau) * math.exp(-t / tau) - tau,
           lambda t: t - tau + tau * math.exp(-t / tau),
           lambda t: math.exp(-t / tau),
           lambda t: (t + tau) * math.exp(-t / tau),
           lambda t: tau * math.exp(-t / tau)]
    q = orc.time_coeffs(dt, tau)
    for k, f in enumerate(fns):
        ref = integrate.quad(f, 0.0, dt, epsabs=0, epsrel=1e-13, limit=200)[0]
        assert abs(q[k] - ref) <= 1e-10 * max(abs(ref), dt * max(dt, tau) * 1e-3)


# ----------------------------------------------------------------- fluxes --

def _frame_n(dim, rng):
    n = rng.normal(size=dim)
    return n / np.linalg.norm(n)


@pytest.mark.parametrize("dim", [2, 3])
def test_gks_uniform_state_gives_euler_flux(orc, dim):
    """f = g for a uniform state: the flux is the Euler flux, W(dt) = W, DF = 1."""
    rng = np.random.default_rng(10 + dim)
    n = _frame_n(dim, rng)
    W = cons(1.1, rng.uniform(-2, 2, dim), 0.7)
    z = np.zeros((dim + 2) * dim)
    for re in (0.0, 500.0):
        F, G, a = orc.gks_point(W, z, W, z, n, 1e-2, dim=dim, reynolds=re, mach=1.5)
        np.testing.assert_allclose(F, euler_flux(W, n), rtol=1e-13, atol=1e-13 * np.abs(W).max())
        np.testing.assert_allclose(G, W, rtol=1e-13, atol=1e-13)
        assert a == 1.0


def _cons_grad(rho, u, p, drho, du, dp, gamma=GAMMA):
    """Cartesian gradients of conservative variables from primitive gradients."""
    dim = len(u)
    g = np.zeros((dim + 2, dim))
    g[0] = drho
    for i in range(dim):
        g[1 + i] = u[i] * drho + rho * du[i]
    g[-1] = dp / (gamma - 1.0) + 0.5 * (u @ u) * drho + rho * (u @ du)
    return g


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("pr", [1.0, 0.72])
def test_gks_navier_stokes_limit(orc, dim, pr):
    """Continuous linear data, dt/tau -> 0: Euler flux minus the Chapman-Enskog
    stress and heat flux with mu = tau p (Eq. ce-ns), heat flux scaled by 1/Pr."""
    rng = np.random.default_rng(20 + dim)
    n = _frame_n(dim, rng)
    rho, p = 1.2, 0.9
    u = rng.uniform(-0.8, 0.8, dim)
    drho, dp = rng.normal(size=dim) * 0.3, rng.normal(size=dim) * 0.3
    du = rng.normal(size=(dim, dim)) * 0.4  # du[i, j] = d u_i / d x_j
    W = cons(rho, u, p)
    g = _cons_grad(rho, u, p, drho, du, dp)
    mach, re, S = 2.0, 100.0, 0.5
    Tinf, T = 1.0 / GAMMA, p / rho
    mu = mach / re * (T / Tinf) ** 1.5 * (Tinf + S * Tinf) / (T + S * Tinf)
    tau = mu / p
    F, _, a = orc.gks_point(W, g.ravel(), W, g.ravel(), n, 1e-6 * tau, dim=dim, reynolds=re,
                            mach=mach, prandtl=pr, sutherland_S_ratio=S)
    K = 2.0 / (GAMMA - 1.0) - dim
    N = dim + K
    divu = np.trace(du)
    sigma = mu * (du + du.T - (2.0 / N) * divu * np.eye(dim))
    cp = (N + 2.0) / 2.0
    dT = dp / rho - p / rho ** 2 * drho
    q = -mu * cp / pr * dT
    ref = euler_flux(W, n).copy()
    ref[1:1 + dim] -= sigma @ n
    ref[-1] += -(sigma @ n) @ u + q @ n
    visc = ref - euler_flux(W, n)
    np.testing.assert_allclose(F - euler_flux(W, n), visc, rtol=2e-5, atol=2e-5 * np.abs(visc).max())
    assert a == 1.0


@pytest.mark.parametrize("dim", [2, 3])
def test_gks_free_transport_limit_is_kfvs(orc, dim):
    """tau >> dt, no slopes: the flux is the collisionless (KFVS) flux of the two states."""
    rng = np.random.default_rng(30 + dim)
    n = _frame_n(dim, rng)
    Wl = cons(1.0, rng.uniform(-1, 1, dim), 0.7)
    Wr = cons(0.6, rng.uniform(-1, 1, dim), 0.4)
    z = np.zeros((dim + 2) * dim)
    dt = 1e-9
    # deviation from the limit is O(dt/tau) = 1e-7; 1 - exp(-dt/tau) loses ~1e-9
    F, _, _ = orc.gks_point(Wl, z, Wr, z, n, dt, dim=dim, tau_c1=1e7, tau_c2=0.0)
    Fk = orc.kfvs_point(Wl, Wr, n, dim=dim)
    np.testing.assert_allclose(F, Fk, rtol=1e-6, atol=1e-6 * np.abs(Fk).max())


def _interface_state_quadrature(Wl, Wr, n, dim):
    """Half-range combination of two Maxwellians (Eq. compatibility2) by quadrature."""
    K = 2.0 / (GAMMA - 1.0) - dim
    out = np.zeros(dim + 2)
    for W, sgn in ((Wl, +1), (Wr, -1)):
        rho = W[0]
        u = W[1:1 + dim] / rho
        p = (GAMMA - 1.0) * (W[-1] - 0.5 * rho * u @ u)
        lam = rho / (2 * p)
        un = u @ n
        f = lambda x, k: x ** k * math.sqrt(lam / math.pi) * math.exp(-lam * (x - un) ** 2)
        lo, hi = (0.0, np.inf) if sgn > 0 else (-np.inf, 0.0)
        m0 = integrate.quad(f, lo, hi, args=(0,), epsrel=1e-13, epsabs=0)[0]
        m1 = integrate.quad(f, lo, hi, args=(1,), epsrel=1e-13, epsabs=0)[0]
        m2 = integrate.quad(f, lo, hi, args=(2,), epsrel=1e-13, epsabs=0)[0]
        ut = u - un * np.asarray(n)
        tt = (dim - 1) / (2 * lam) + ut @ ut + K / (2 * lam)
        out[0] += rho * m0
        out[1:1 + dim] += rho * (m1 * np.asarray(n) + m0 * ut)
        out[-1] += rho * 0.5 * (m2 + m0 * tt)
    return out


@pytest.mark.parametrize("dim", [2, 3])
def test_gks_collision_dominated_limit(orc, dim):
    """tau -> 0, no slopes: the flux is the Euler flux of the interface equilibrium W^c."""
    rng = np.random.default_rng(40 + dim)
    n = _frame_n(dim, rng)
    Wl = cons(1.0, rng.uniform(-1, 1, dim), 0.7)
    Wr = cons(0.8, rng.uniform(-1, 1, dim), 0.9)
    z = np.zeros((dim + 2) * dim)
    F, G, _ = orc.gks_point(Wl, z, Wr, z, n, 1.0, dim=dim, tau_c1=1e-12, tau_c2=0.0)
    Wc = _interface_state_quadrature(Wl, Wr, n, dim)
    np.testing.assert_allclose(G, Wc, rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(F, euler_flux(Wc, n), rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("dim", [2, 3])
def test_kfvs_equal_states_is_euler_flux(orc, dim):
    rng = np.random.default_rng(50 + dim)
    n = _frame_n(dim, rng)
    W = cons(0.9, rng.uniform(-3, 3, dim), 1.1)
    np.testing.assert_allclose(orc.kfvs_point(W, W, n, dim=dim), euler_flux(W, n), rtol=1e-13, atol=1e-13)


def test_discontinuity_feedback_closed_form(orc):
    """alpha = 1/(1+D^2) with D from pressure and Mach jumps (Sec. 3.3)."""
    n = np.array([0.6, 0.8])
    t = np.array([-0.8, 0.6])
    rl, pl, rr, pr_ = 1.0, 1.0, 0.5, 0.3
    ul = 0.4 * n + 0.2 * t
    ur = -0.1 * n + 0.7 * t
    Wl, Wr = cons(rl, ul, pl), cons(rr, ur, pr_)
    cl, cr = math.sqrt(GAMMA * pl / rl), math.sqrt(GAMMA * pr_ / rr)
    D = abs(pl - pr_) / pl + abs(pl - pr_) / pr_ + (0.4 / cl + 0.1 / cr) ** 2 + (0.2 / cl - 0.7 / cr) ** 2
    z = np.zeros(8)
    _, _, a = orc.gks_point(Wl, z, Wr, z, n, 1e-3)
    assert a == pytest.approx(1.0 / (1.0 + D * D), rel=1e-13)


@pytest.mark.parametrize("dim", [2, 3])
def test_slip_wall_mirror_flux_has_no_mass_or_energy_flux(orc, dim):
    rng = np.random.default_rng(60 + dim)
    n = _frame_n(dim, rng)
    W = cons(1.1, rng.uniform(-1, 1, dim), 0.8)
    g = rng.normal(size=(dim + 2) * dim) * 0.2
    Wg, gg = orc.ghost(2, W, g, n, dim=dim)
    # ghost is the mirror image: normal momentum flips, the rest is kept
    un = W[1:1 + dim] @ n
    np.testing.assert_allclose(Wg[1:1 + dim], W[1:1 + dim] - 2 * un * n, rtol=1e-14, atol=1e-15)
    for re in (0.0, 300.0):
        F, _, _ = orc.gks_point(W, g, Wg, gg, n, 1e-2, dim=dim, reynolds=re, mach=0.5)
        scale = np.abs(F).max()
        assert abs(F[0]) <= 1e-14 * scale
        assert abs(F[-1]) <= 1e-13 * scale


def test_farfield_ghost_of_free_stream_is_free_stream(orc):
    for mach in (0.38, 8.0):
        Winf = cons(1.0, [mach, 0.0], 1.0 / GAMMA)
        for ang in np.linspace(0, 2 * np.pi, 9):
            n = np.array([math.cos(ang), math.sin(ang)])
            Wg, _ = orc.ghost(1, Winf, None, n, mach=mach)
            np.testing.assert_allclose(Wg, Winf, rtol=1e-14, atol=1e-14)


def test_farfield_subsonic_branch_follows_free_stream_direction(orc):
    """Riemann invariants fix the boundary normal velocity and sound speed; the
    entropy (and tangential velocity) come from the interior where the free stream
    leaves through the face (u_inf . n > 0) and from the free stream elsewhere,
    whatever the sign of the local normal velocity."""
    G, mach = 1.4, 0.5
    for ang, outflow in ((80.0, True), (100.0, False)):
        n = np.array([np.cos(np.radians(ang)), np.sin(np.radians(ang))])
        # interior: the free stream's sound speed but another entropy, moving against
        # the free stream's normal direction
        rho, p = 1.2, 1.2 / G
        u = np.array([mach, 0.0]) - (0.2 if outflow else -0.2) * n
        W = np.array([rho, rho * u[0], rho * u[1], p / (G - 1) + 0.5 * rho * u @ u])
        Wg, _ = orc.ghost(1, W, None, n, mach=mach)
        ub = 0.5 * ((u @ n + 2 * np.sqrt(G * p / rho) / (G - 1)) + (mach * n[0] - 2 * np.sqrt(G / G * 1.0) / (G - 1)))
        assert (ub > 0) != outflow           # the local normal velocity points the other way
        pg = (G - 1) * (Wg[3] - 0.5 * (Wg[1] ** 2 + Wg[2] ** 2) / Wg[0])
        s_ghost, s_in, s_inf = pg / Wg[0] ** G, p / rho ** G, (1.0 / G)
        assert s_ghost == pytest.approx(s_in if outflow else s_inf, rel=1e-12)
        assert (Wg[1:3] / Wg[0]) @ n == pytest.approx(ub, rel=1e-12)


def test_isothermal_ghost_sets_wall_temperature_and_no_slip(orc):
    W = cons(1.3, [0.2, -0.1], 0.9)
    n = np.array([0.0, -1.0])
    Wg, _ = orc.ghost(3, W, None, n, wall_T_ratio=1.0)
    Tw = 1.0 / GAMMA
    rho_g = Wg[0]
    ug = Wg[1:3] / rho_g
    pg = (GAMMA - 1) * (Wg[3] - 0.5 * rho_g * ug @ ug)
    assert 0.5 * (0.9 / 1.3 + pg / rho_g) == pytest.approx(Tw, rel=1e-14)
    np.testing.assert_allclose(0.5 * (W[1:3] / W[0] + ug), 0.0, atol=1e-15)
    assert pg == pytest.approx(0.9, rel=1e-14)
