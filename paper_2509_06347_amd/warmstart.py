"""Warm start of steady cylinder solves from the BF16-MFMA surrogate network.

Data: converged steady solutions produced by the batched V-cycle solver.
Features per fine cell: Mach, log10 Re, centroid x, y and the distance to the
nearest wall-face centre, computed on the device by `cgks_mlp_features` — the
same kernel `cgks_init_from_mlp` evaluates before inference.
Targets per cell: log(rho / rho_inf), u / U_inf, v / U_inf, log(p / p_inf).
Features and targets are standardised with the training set's mean and
standard deviation.  Training runs on the GPU through `cgks_mlp_train_step`
(Adam, cosine-decayed learning rate, fixed-order reductions).

The features, the network's training and inference and the solves run in
the library; this module draws problems and mini-batch indices, standardises
the data (mean and standard deviation of the training set) and transforms
the converged states into targets.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import cgks

GAMMA = 1.4


def targets(W, mach):
    """Raw targets [n, 4] from conservative states [n, 4]."""
    rho = W[:, 0]
    u, v = W[:, 1] / rho, W[:, 2] / rho
    p = (GAMMA - 1.0) * (W[:, 3] - 0.5 * rho * (u * u + v * v))
    return np.column_stack([np.log(rho), u / mach, v / mach, np.log(p * GAMMA)])


@dataclass
class Problem:
    mach: float
    reynolds: float
    mesh: object


def draw_problems(seed, n, mesh_fn, mach=(0.1, 0.3), reynolds=(30.0, 40.0), mesh_seed0=5000):
    """n problems with Mach uniform and Re log-uniform in the given ranges."""
    rng = np.random.default_rng(seed)
    ms = rng.uniform(*mach, size=n)
    rs = np.exp(rng.uniform(math.log(reynolds[0]), math.log(reynolds[1]), size=n))
    return [Problem(float(m), float(r), mesh_fn(mesh_seed0 + k)) for k, (m, r) in enumerate(zip(ms, rs))]


def batched_solve(problems, tol, max_cycles, init=None, n_levels=3, **params):
    """Solve the problems together (one disjoint-union batch).  init(k, solver)
    sets problem k's initial state (default: free stream).  Returns the solvers
    (holding the final states), per-problem cycles to tol, statuses and the
    wall time from the first initialisation to the end of the solve."""
    import torch
    solvers = [cgks.Solver(p.mesh, n_levels=n_levels, mach=p.mach, reynolds=p.reynolds, **params)
               for p in problems]
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k, s in enumerate(solvers):
        if init is None:
            s.init_freestream()
        else:
            init(k, s)
    batch = cgks.Batch(solvers)
    rc, cycles, status = batch.solve(tol=tol, max_cycles=max_cycles)
    batch.sync_states()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    batch.close()
    return solvers, cycles, status, wall


def dataset(problems, solvers, status):
    """Features and targets of the converged problems."""
    X, Y = [], []
    for p, s, st in zip(problems, solvers, status):
        if st != cgks.OK:
            continue
        W, _, _ = s.get_state()
        X.append(s.mlp_features().astype(np.float64))
        Y.append(targets(W, p.mach))
    return np.concatenate(X), np.concatenate(Y)


@dataclass
class Scaling:
    fmean: np.ndarray
    fstd: np.ndarray
    tmean: np.ndarray
    tstd: np.ndarray
    flo: np.ndarray = None      # training range of the raw features
    fhi: np.ndarray = None

    @classmethod
    def fit(cls, X, Y):
        fs = X.std(axis=0)
        fs[fs == 0] = 1.0
        ts = Y.std(axis=0)
        ts[ts == 0] = 1.0
        return cls(X.mean(axis=0), fs, Y.mean(axis=0), ts, X.min(axis=0), X.max(axis=0))


def train(net, X, Y, scaling, steps, batch=16384, lr=1e-3, seed=0, log_every=0):
    """Adam on standardised data with a cosine-decayed learning rate; the data
    stay in device memory and mini-batches are drawn without replacement per
    epoch.  Returns the per-step losses."""
    import torch
    Xs = torch.from_numpy(((X - scaling.fmean) / scaling.fstd).astype(np.float32)).cuda()
    Ys = torch.from_numpy(((Y - scaling.tmean) / scaling.tstd).astype(np.float32)).cuda()
    n = Xs.shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    pos, losses = 0, []
    for it in range(steps):
        if pos + batch > n:
            perm, pos = rng.permutation(n), 0
        idx = torch.from_numpy(perm[pos:pos + batch]).cuda()
        pos += batch
        xb = Xs.index_select(0, idx).contiguous()
        yb = Ys.index_select(0, idx).contiguous()
        a = lr * 0.5 * (1.0 + math.cos(math.pi * it / steps))
        losses.append(net.train_step(xb, yb, max(a, 1e-3 * lr)))
        if log_every and it % log_every == 0:
            print(f"  step {it:5d} loss {losses[-1]:.4e}", flush=True)
    return losses


def warm_init(net, scaling):
    """An init(k, solver) for batched_solve that warm-starts from the network;
    cells whose features leave the training range take the free stream."""
    if scaling.flo is not None:
        net.set_range(scaling.flo, scaling.fhi)

    def init(k, solver):
        net.init_solver(solver, scaling.fmean, scaling.fstd, scaling.tmean, scaling.tstd)
    return init
