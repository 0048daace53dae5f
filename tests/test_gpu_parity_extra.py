"""Parity at size and for the additions, through the C ABI against the oracle.

* A 3-D Kuhn sphere shell of 380,928 tetrahedra (16 x 8 x 8 grid, two
  Freudenthal refinements; the C3 family at an eighth of its size), Mach 6:
  every cell's fine residual, evolved slopes and DF at a perturbed state, then
  one V-cycle from that state.
* The FP32 coarse correction (precision = MIXED) against the FP64 oracle along
  a V-cycle trajectory: the first norm is computed before any coarse work and
  agrees to FP64 rounding; afterwards the states differ by the FP32 rounding
  of the coarse corrections (relative ~6e-8 per operation, accumulated over
  6 sweeps on 2 levels per cycle), bounded here by 1e-6 of the state.
* Each member of a batched solve (uneven meshes, different Mach, Reynolds
  number and incidence; all Navier-Stokes, as one batch must be) against the
  oracle's single solve.

The printed figures are the observed errors."""
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


def _shell_state(o, mach, seed, amp=0.02, slope=1e-3):
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
    return W, slope * rng.standard_normal((len(V), 5, 3)), rng.uniform(0.5, 1.0, len(V))


def test_large_kuhn_shell_residual_and_vcycle(cg, orc):
    mesh = sm.sphere_shell_kuhn(16, 8, 8, nref=2)
    assert mesh.n_cells >= 300_000
    params = dict(dim=3, mach=6.0, cfl_ramp=10)
    print(f"[case] Kuhn shell 16x8x8 nref 2: {mesh.n_cells} tetrahedra, {params}", flush=True)
    g = cg.Solver(mesh, n_levels=3, **params)
    o = orc.Oracle(mesh, n_levels=3, **params)
    assert g.sizes == [tuple(s) for s in o.sizes]
    for l in (1, 2):
        cgc, ncg = g.coloring(l)
        coc, nco = o.coloring(l)
        assert ncg == nco and np.array_equal(cgc, coc)
    W, grad, alpha = _shell_state(o, 6.0, seed=11)
    for s in (g, o):
        s.set_state(W, grad, alpha)
    Rg, gg, ag = g.residual(0)
    Ro, go, ao = o.residual(0)
    err = np.abs(Rg - Ro).max()
    print(f"residual: max err / max |R| = {err / np.abs(Ro).max():.2e}, "
          f"/ flux-sum scale = {err / o.flux_scale():.2e}", flush=True)
    assert err <= 1e-12 * np.abs(Ro).max()
    assert np.abs(gg - go).max() <= 1e-11 * np.abs(go).max()
    np.testing.assert_allclose(ag, ao, rtol=1e-10, atol=1e-13)
    # one V-cycle from the perturbed state (slopes zero, DF one)
    for s in (g, o):
        s.set_state(W, None, None)
    ng = g.vcycle()
    no = o.vcycle()
    Wg, _, _ = g.get_state()
    Wo, _, _ = o.get_state()
    werr = np.abs(Wg - Wo).max() / np.abs(Wo).max()
    print(f"V-cycle: norm {ng:.6e} vs {no:.6e}, state err {werr:.2e}", flush=True)
    np.testing.assert_allclose(ng, no, rtol=1e-10)
    assert werr <= 1e-10
    assert g.stats()[1] == o.stats()[1]


def test_fp32_correction_cycle_against_fp64_oracle(cg, orc):
    mesh = sm.annulus(32, 8, jitter=0.15, seed=0, nref=2, wall_tag=sm.ISOTHERMAL)
    prm = dict(mach=0.15, reynolds=40.0)
    g = cg.Solver(mesh, n_levels=3, precision=cg.MIXED, **prm)
    o = orc.Oracle(mesh, n_levels=3, **prm)
    for s in (g, o):
        s.init_freestream()
    ng = g.run_cycles(6)
    no = np.array([o.vcycle() for _ in range(6)])
    Wg, _, _ = g.get_state()
    Wo, _, _ = o.get_state()
    werr = np.abs(Wg - Wo).max() / np.abs(Wo).max()
    nerr = np.abs(ng - no).max() / np.abs(no).max()
    print(f"FP32 correction vs FP64 oracle after 6 cycles: state {werr:.2e}, norms {nerr:.2e}", flush=True)
    np.testing.assert_allclose(ng[0], no[0], rtol=1e-12)
    assert nerr <= 1e-5
    assert werr <= 1e-6


def test_batch_member_against_oracle(cg, orc):
    specs = [(sm.annulus(12, 4, jitter=0.1, seed=1, nref=2, wall_tag=sm.ISOTHERMAL), dict(mach=0.3, reynolds=40.0)),
             (sm.annulus(13, 5, jitter=0.2, seed=3, nref=2, wall_tag=sm.ISOTHERMAL), dict(mach=0.7, reynolds=500.0,
                                                                                         aoa_deg=12.0))]
    members, oracles = [], []
    for mesh, p in specs:
        s = cg.Solver(mesh, n_levels=3, **p)
        s.init_freestream()
        members.append(s)
        o = orc.Oracle(mesh, n_levels=3, **p)
        o.init_freestream()
        oracles.append(o)
    batch = cg.Batch(members)
    hist = batch.run_cycles(4)
    batch.sync_states()
    for b, o in enumerate(oracles):
        no = np.array([o.vcycle() for _ in range(4)])
        Wb, _, _ = members[b].get_state()
        Wo, _, _ = o.get_state()
        werr = np.abs(Wb - Wo).max() / np.abs(Wo).max()
        print(f"batch member {b}: state err {werr:.2e}", flush=True)
        np.testing.assert_allclose(hist[b], no, rtol=1e-10)
        assert werr <= 1e-10
