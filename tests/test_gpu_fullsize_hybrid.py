"""GPU (HIP) vs CPU oracle on the hybrid-mesh workload at full size.

The viscous Mach 0.5 box of 1,201,412 hybrid cells (tetrahedra, pyramids,
prisms and hexahedra; isothermal wall at z = 0), run as the benchmark runs
it: the solver on torch's current stream, the free-stream start with the
velocity ramped to zero at the wall and the 10-cycle CFL ramp, 10 V-cycles,
then the autotuner's launch shapes.  At the resulting state the GPU computes
the whole fine residual; the oracle computes the residual, evolved slopes
and DF of a sample of cells (2,000 next to the wall, 1,000 next to the far
field and 10,000 random cells) with the same routines as its full residual,
and the time steps of every cell.  Bars as in the other residual parity
tests.
"""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(400)
def test_hybrid_fullsize_sampled_residual_parity(orc):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import bench
    from paper_2509_06347_amd import cgks
    t0 = time.perf_counter()
    mesh, params = bench.workload("hybrid_box_ns_mach0.5_1.2M")
    print(f"[case] full-size hybrid: cells={mesh.n_cells} {mesh.info} (mesh {time.perf_counter() - t0:.0f} s)",
          flush=True)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    g = cgks.Solver(mesh, n_levels=3, stream=stream.cuda_stream, **params)
    print(f"[case] library set-up {time.perf_counter() - t0:.0f} s, levels {g.sizes}", flush=True)
    bench.initial_state(g, mesh, params)
    g.run_cycles(10)
    shapes = g.autotune()
    print(f"[case] autotuned launch shapes {shapes}, coarse {g.coarse_shapes()}", flush=True)
    W, grad, alpha = g.get_state()
    Rg, gg, ag = g.residual(0)
    dg, _ = g.time_steps(0)

    t0 = time.perf_counter()
    o = orc.Oracle(mesh, n_levels=1, **params)
    o.set_state(W, grad, alpha)
    print(f"[case] oracle set-up {time.perf_counter() - t0:.0f} s", flush=True)
    rng = np.random.default_rng(23)
    _, C = o.cell_geometry(0)
    near_wall = np.nonzero(C[:, 2] < 0.01)[0]
    near_far = np.nonzero(C[:, 2] > 0.99)[0]
    cells = np.unique(np.concatenate([rng.choice(near_wall, 2000, replace=False),
                                      rng.choice(near_far, 1000, replace=False),
                                      rng.choice(mesh.n_cells, 10000, replace=False)]))
    t0 = time.perf_counter()
    Ro, go, ao = o.residual_cells(cells)
    print(f"[case] oracle sampled residual of {len(cells)} cells {time.perf_counter() - t0:.0f} s", flush=True)
    scale = np.abs(Rg).max()
    err = np.abs(Rg[cells] - Ro).max()
    print(f"residual: max |dR| / max |R| = {err / scale:.2e}", flush=True)
    assert err <= 1e-12 * scale
    gerr = np.abs(gg[cells] - go).max() / np.abs(go).max()
    print(f"slopes: max |dg| / max |g| = {gerr:.2e}", flush=True)
    assert gerr <= 1e-11
    aerr = np.abs(ag[cells] - ao).max()
    print(f"DF: max |da| = {aerr:.2e}", flush=True)
    np.testing.assert_allclose(ag[cells], ao, rtol=1e-12, atol=1e-13)
    do, _ = o.time_steps(0)
    np.testing.assert_allclose(dg, do, rtol=1e-13)
