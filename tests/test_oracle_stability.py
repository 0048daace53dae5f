"""Linear stability of the explicit fine step (Eq. smo with the direct slope
evolution of Sec. 2.4) at an exact steady state, a uniform stream through a
small far-field square.

The Jacobian of one step x -> x' (x = cell averages and slopes) is built by
central finite differences of the oracle and its eigenvalues are taken.
Findings pinned here (they explain why the steady inviscid cases stall):
  * with the collision-time coefficient tau = 0.01 dt (the Euler reading) the
    step has a real eigenvalue above 1; its excess grows in proportion to the
    explicit CFL number, so it is an instability of the spatial operator (the
    compact reconstruction fed by the evolved slopes), not of the time step;
    the mode is mostly slopes and alternates from row to row across the stream;
  * with the slope map alone (cell averages held fixed) the same step
    contracts quickly, so the growth lives in the coupling of averages and
    slopes;
  * tau = 0.1 dt adds enough dissipation to make the step contract.
Linear weights are used so that the map is smooth at the free stream."""
import numpy as np
import pytest

import synthmesh as sm


def _step_jacobian(orc, n=6, eps=1e-7, **kw):
    mesh = sm.structured_square(n, jitter=0.1, seed=3)
    p = dict(mach=0.38, slope_relax=1.0, weno_gamma_large=1.0)
    p.update(kw)
    o = orc.Oracle(mesh, n_levels=1, **p)
    o.init_freestream()
    W0, g0, _ = o.get_state()
    nW = W0.size
    x0 = np.concatenate([W0.ravel(), g0.ravel()])

    def step(x):
        o.set_state(x[:nW].reshape(W0.shape), x[nW:].reshape(g0.shape))
        o.vcycle()
        W, g, _ = o.get_state()
        return np.concatenate([W.ravel(), g.ravel()])

    assert np.abs(step(x0) - x0).max() < 1e-13          # an exact fixed point
    J = np.empty((x0.size, x0.size))
    for k in range(x0.size):
        e = np.zeros(x0.size)
        e[k] = eps
        J[:, k] = (step(x0 + e) - step(x0 - e)) / (2 * eps)
    return J, nW


@pytest.mark.slow
def test_explicit_step_unstable_with_small_collision_time(orc):
    rad = {}
    for cfl in (0.5, 0.25):
        J, nW = _step_jacobian(orc, cfl_exp=cfl, tau_c1=0.01)
        lam, vec = np.linalg.eig(J)
        k = np.argmax(np.abs(lam))
        rad[cfl] = lam[k]
        if cfl == 0.5:
            v = np.abs(vec[:, k])
            assert abs(lam[k].imag) < 1e-9                 # a real, growing mode
            assert np.linalg.norm(v[nW:]) > 0.9            # carried by the slopes
            # the slope map alone contracts (averages frozen)
            Jg = J[nW:, nW:]
            assert np.abs(np.linalg.eigvals(Jg)).max() < 0.9
    assert rad[0.5].real > 1.0005 and rad[0.25].real > 1.0002
    # growth proportional to the step: (lambda - 1) / CFL about the same
    g1, g2 = (rad[0.5].real - 1) / 0.5, (rad[0.25].real - 1) / 0.25
    assert 0.6 < g1 / g2 < 1.4


@pytest.mark.slow
def test_explicit_step_contracts_with_larger_collision_time(orc):
    J, _ = _step_jacobian(orc, cfl_exp=0.5, tau_c1=0.1)
    assert np.abs(np.linalg.eigvals(J)).max() < 0.9995
