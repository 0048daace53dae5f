"""ctypes wrapper of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
import this module.  The product package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

FARFIELD, SLIP, ISOTHERMAL, ADIABATIC = 1, 2, 3, 4


class Params(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("gamma", C.c_double), ("prandtl", C.c_double),
        ("mach", C.c_double), ("aoa_deg", C.c_double), ("reynolds", C.c_double),
        ("wall_T_ratio", C.c_double), ("sutherland_S_ratio", C.c_double),
        ("cfl_exp", C.c_double), ("cfl_imp", C.c_double), ("n_levels", C.c_int),
        ("n_pre_fine", C.c_int), ("n_post", C.c_int), ("n_sweeps", C.c_int),
        ("df_relax", C.c_int), ("df_prolong", C.c_int), ("precision", C.c_int),
        ("tau_c1", C.c_double), ("tau_c2", C.c_double),
        ("weno_gamma_large", C.c_double), ("weno_eps", C.c_double),
        ("lusgs_omega", C.c_double), ("skew_limit", C.c_double),
        ("slope_relax", C.c_double), ("update_limit", C.c_double), ("cfl_ramp", C.c_int),
        ("relax_beta", C.c_double), ("shared_residual", C.c_int), ("slip_wall_p1", C.c_int),
    ]


# The oracle's own defaults: its readings of the paper where the paper is silent.
DEFAULTS = dict(dim=2, gamma=1.4, prandtl=0.72, mach=0.38, aoa_deg=0.0, reynolds=0.0,
                wall_T_ratio=1.0, sutherland_S_ratio=0.5, cfl_exp=0.5, cfl_imp=10.0,
                n_levels=3, n_pre_fine=1, n_post=0, n_sweeps=6, df_relax=1, df_prolong=1,
                precision=0, tau_c1=0.01, tau_c2=1.0, weno_gamma_large=0.95,
                weno_eps=1e-14, lusgs_omega=1.0, skew_limit=0.2, slope_relax=0.3,
                update_limit=0.5, cfl_ramp=0, relax_beta=0.5, shared_residual=0, slip_wall_p1=0)


class OrcMesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_nodes", C.c_int), ("coords", C.POINTER(C.c_double)),
                ("n_cells", C.c_int), ("cell_nodes", C.POINTER(C.c_int32)),
                ("n_bfaces", C.c_int), ("bface_nodes", C.POINTER(C.c_int32)),
                ("bface_tag", C.POINTER(C.c_int32)),
                ("cell_offsets", C.POINTER(C.c_int32)), ("bface_offsets", C.POINTER(C.c_int32))]


def build():
    subprocess.run(["sh", os.path.join(_HERE, "build.sh")], check=True)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            build()
        _LIB = C.CDLL(path)
        _LIB.orc_last_error.restype = C.c_char_p
    return _LIB


def set_threads(n):
    """OpenMP threads of the oracle's loops (results are bitwise independent of it)."""
    if lib().orc_set_threads(int(n)) != 0:
        raise ValueError("thread count must be >= 1")


def get_threads():
    return int(lib().orc_get_threads())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def make_params(**kw):
    d = dict(DEFAULTS)
    d.update(kw)
    p = Params()
    for k, v in d.items():
        setattr(p, k, v)
    return p


class OracleError(RuntimeError):
    pass


class Oracle:
    """One oracle solver context on a mesh from :mod:`synthmesh`."""

    def __init__(self, mesh, n_levels=3, use_parents=True, **params):
        L = lib()
        params.setdefault("dim", mesh.dim)
        params.setdefault("n_levels", n_levels)
        self.p = make_params(**params)
        self.dim = mesh.dim
        self.nvar = mesh.dim + 2
        ctx = C.c_void_p()
        self._chk(L.orc_create(C.byref(self.p), C.byref(ctx)), None)
        self.ctx = ctx
        self._keep = [np.ascontiguousarray(mesh.coords, dtype=np.float64),
                      np.ascontiguousarray(mesh.cells, dtype=np.int32),
                      np.ascontiguousarray(mesh.bfaces, dtype=np.int32),
                      np.ascontiguousarray(mesh.btags, dtype=np.int32)]
        m = OrcMesh(mesh.dim, mesh.n_nodes, _dp(self._keep[0]), mesh.n_cells, _ip(self._keep[1]),
                    len(mesh.btags), _ip(self._keep[2]), _ip(self._keep[3]))
        if getattr(mesh, "cell_offsets", None) is not None:
            self._keep += [np.ascontiguousarray(mesh.cell_offsets, dtype=np.int32),
                           np.ascontiguousarray(mesh.bface_offsets, dtype=np.int32)]
            m.cell_offsets, m.bface_offsets = _ip(self._keep[4]), _ip(self._keep[5])
        par = (C.POINTER(C.c_int32) * max(n_levels - 1, 1))()
        pk = []
        for l in range(n_levels - 1):
            if use_parents and l < len(mesh.parents):
                a = np.ascontiguousarray(mesh.parents[l], dtype=np.int32)
                pk.append(a)
                par[l] = _ip(a)
            else:
                par[l] = C.POINTER(C.c_int32)()
        self._keep += pk
        self._chk(L.orc_mesh_setup(ctx, C.byref(m), n_levels, par))
        self.n_levels = n_levels
        self.sizes = []
        for l in range(n_levels):
            nc, nf = C.c_int(), C.c_int()
            L.orc_level_size(ctx, l, C.byref(nc), C.byref(nf))
            self.sizes.append((nc.value, nf.value))

    def _chk(self, rc, ctx=0):
        if rc < 0:
            msg = ""
            if ctx is not None and getattr(self, "ctx", None):
                msg = lib().orc_last_error(self.ctx).decode()
            raise OracleError(f"oracle error {rc}: {msg}")
        return rc

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                lib().orc_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # geometry ------------------------------------------------------------
    def cell_geometry(self, level=0):
        n = self.sizes[level][0]
        V = np.zeros(n)
        Cc = np.zeros((n, self.dim))
        self._chk(lib().orc_cell_geometry(self.ctx, level, _dp(V), _dp(Cc)))
        return V, Cc

    def face_geometry(self, level=0):
        nf = self.sizes[level][1]
        LR = np.zeros((nf, 2), dtype=np.int32)
        tag = np.zeros(nf, dtype=np.int32)
        n = np.zeros((nf, self.dim))
        S = np.zeros(nf)
        xc = np.zeros((nf, self.dim))
        self._chk(lib().orc_face_geometry(self.ctx, level, _ip(LR), _ip(tag), _dp(n), _dp(S), _dp(xc)))
        return dict(LR=LR, tag=tag, n=n, S=S, xc=xc)

    def face_quadrature(self):
        nf = self.sizes[0][1]
        ngp = np.zeros(nf, dtype=np.int32)
        gp = np.zeros((nf, 4, self.dim))
        w = np.zeros((nf, 4))
        self._chk(lib().orc_face_quadrature(self.ctx, _ip(ngp), _dp(gp), _dp(w)))
        return ngp, gp, w

    def coloring(self, level):
        n = self.sizes[level][0]
        col = np.zeros(n, dtype=np.int32)
        nc = C.c_int32()
        self._chk(lib().orc_coloring(self.ctx, level, _ip(col), C.byref(nc)))
        return col, nc.value

    def agglomerate(self, level=0):
        n = self.sizes[level][0]
        agg = np.zeros(n, dtype=np.int32)
        nc = C.c_int32()
        self._chk(lib().orc_agglomerate(self.ctx, level, _ip(agg), C.byref(nc)))
        return agg, nc.value

    # state ---------------------------------------------------------------
    def init_freestream(self):
        self._chk(lib().orc_init_freestream(self.ctx))

    def set_state(self, W, grad=None, alpha=None):
        W = np.ascontiguousarray(W, dtype=np.float64)
        g = None if grad is None else np.ascontiguousarray(grad, dtype=np.float64)
        a = None if alpha is None else np.ascontiguousarray(alpha, dtype=np.float64)
        self._chk(lib().orc_set_state(self.ctx, _dp(W), _dp(g) if g is not None else None,
                                      _dp(a) if a is not None else None))

    def get_state(self):
        n = self.sizes[0][0]
        W = np.zeros((n, self.nvar))
        g = np.zeros((n, self.nvar, self.dim))
        a = np.zeros(n)
        self._chk(lib().orc_get_state(self.ctx, _dp(W), _dp(g), _dp(a)))
        return W, g, a

    def get_level_state(self, level):
        n = self.sizes[level][0]
        W, W0, F = (np.zeros((n, self.nvar)) for _ in range(3))
        a = np.zeros(n)
        self._chk(lib().orc_get_level_state(self.ctx, level, _dp(W), _dp(W0), _dp(F), _dp(a)))
        return W, W0, F, a

    def set_level_state(self, level, W=None, W0=None, F=None, alpha=None):
        arrs = [None if x is None else np.ascontiguousarray(x, dtype=np.float64) for x in (W, W0, F, alpha)]
        self._chk(lib().orc_set_level_state(self.ctx, level, *[(_dp(a) if a is not None else None) for a in arrs]))

    # solver --------------------------------------------------------------
    def residual(self, level=0):
        n = self.sizes[level][0]
        R = np.zeros((n, self.nvar))
        g = np.zeros((n, self.nvar, self.dim))
        a = np.zeros(n)
        self._chk(lib().orc_residual(self.ctx, level, _dp(R), _dp(g), _dp(a)))
        return R, g, a

    def residual_cells(self, cells):
        """Fine residual, evolved slopes and DF of the listed cells only (the
        same values as residual(0) for those rows)."""
        idx = np.ascontiguousarray(cells, dtype=np.int32)
        m = len(idx)
        R = np.zeros((m, self.nvar))
        g = np.zeros((m, self.nvar, self.dim))
        a = np.zeros(m)
        self._chk(lib().orc_residual_cells(self.ctx, _ip(idx), m, _dp(R), _dp(g), _dp(a)))
        return R, g, a

    def time_steps(self, level=0):
        n = self.sizes[level][0]
        de, di = np.zeros(n), np.zeros(n)
        self._chk(lib().orc_time_steps(self.ctx, level, _dp(de), _dp(di)))
        return de, di

    def smooth(self, level, n):
        self._chk(lib().orc_smooth(self.ctx, level, n))

    def smooth_sequential(self, level, n):
        self._chk(lib().orc_smooth_sequential(self.ctx, level, n))

    def restrict(self, level):
        self._chk(lib().orc_restrict(self.ctx, level))

    def prolong(self, level):
        self._chk(lib().orc_prolong(self.ctx, level))

    def vcycle(self):
        nrm = C.c_double()
        rc = self._chk(lib().orc_vcycle(self.ctx, C.byref(nrm)))
        return nrm.value

    def solve(self, tol=1e-10, max_cycles=1000):
        hist = np.zeros(max_cycles)
        ncyc = C.c_int()
        rc = self._chk(lib().orc_solve(self.ctx, C.c_double(tol), max_cycles, C.byref(ncyc), _dp(hist), max_cycles))
        return rc, hist[:ncyc.value]

    def flux_scale(self):
        """max over cells and components of sum_f |S_f F_f| (the faces of the
        cell) from the last fine residual: the scale the residual cancels from."""
        nf = self.sizes[0][1]
        F = np.zeros((nf, self.nvar))
        self._chk(lib().orc_face_fluxes(self.ctx, _dp(F)))
        LR = np.zeros((nf, 2), dtype=np.int32)
        self._chk(lib().orc_face_geometry(self.ctx, 0, _ip(LR), None, None, None, None))
        acc = np.zeros((self.sizes[0][0], self.nvar))
        np.add.at(acc, LR[:, 0], np.abs(F))
        inner = LR[:, 1] >= 0
        np.add.at(acc, LR[inner, 1], np.abs(F[inner]))
        return float(acc.max())

    def stats(self):
        a, b = C.c_int64(), C.c_int64()
        lib().orc_stats(self.ctx, C.byref(a), C.byref(b))
        return a.value, b.value

    def recon_eval(self, cell, x):
        nv = self.nvar
        W, g, p2, p1, w = np.zeros(nv), np.zeros((nv, self.dim)), np.zeros(nv), np.zeros(nv), np.zeros(nv)
        xx = np.ascontiguousarray(x, dtype=np.float64)
        self._chk(lib().orc_recon_eval(self.ctx, cell, _dp(xx), _dp(W), _dp(g), _dp(p2), _dp(p1), _dp(w)))
        return W, g, p2, p1, w

    def recon_indicators(self, cell):
        """beta_0, beta_1, the DF-scaled Green-Gauss gradient [nvar, dim] and the
        large-stencil weight of one cell's reconstruction (Sec. 3)."""
        nv = self.nvar
        b0, b1, g1, w = np.zeros(nv), np.zeros(nv), np.zeros((nv, self.dim)), np.zeros(nv)
        self._chk(lib().orc_recon_indicators(self.ctx, cell, _dp(b0), _dp(b1), _dp(g1), _dp(w)))
        return b0, b1, g1, w


# point functions ------------------------------------------------------------

def moments(U, lam, rng, nmax=11):
    out = np.zeros(nmax + 1)
    rc = lib().orc_moments(C.c_double(U), C.c_double(lam), rng, nmax, _dp(out))
    if rc:
        raise OracleError(rc)
    return out


def time_coeffs(dt, tau):
    q = np.zeros(6)
    if lib().orc_time_coeffs(C.c_double(dt), C.c_double(tau), _dp(q)):
        raise OracleError("time_coeffs")
    return q


def moment_solve(W, b, **params):
    p = make_params(**params)
    W = np.ascontiguousarray(W, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    a = np.zeros(p.dim + 2)
    lib().orc_moment_solve(C.byref(p), _dp(W), _dp(b), _dp(a))
    return a


def gks_point(Wl, gl, Wr, gr, n, dt, **params):
    p = make_params(**params)
    nv = p.dim + 2
    args = [np.ascontiguousarray(x, dtype=np.float64) for x in (Wl, gl, Wr, gr, n)]
    F, G, a = np.zeros(nv), np.zeros(nv), C.c_double()
    lib().orc_gks_point(C.byref(p), *[_dp(x) for x in args], C.c_double(dt), _dp(F), _dp(G), C.byref(a))
    return F, G, a.value


def kfvs_point(Wl, Wr, n, **params):
    p = make_params(**params)
    args = [np.ascontiguousarray(x, dtype=np.float64) for x in (Wl, Wr, n)]
    F = np.zeros(p.dim + 2)
    lib().orc_kfvs_point(C.byref(p), *[_dp(x) for x in args], _dp(F))
    return F


def ghost(tag, W, g, n, **params):
    p = make_params(**params)
    nv = p.dim + 2
    W = np.ascontiguousarray(W, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    Wg = np.zeros(nv)
    if g is None:
        lib().orc_ghost(C.byref(p), tag, _dp(W), None, _dp(n), _dp(Wg), None)
        return Wg, None
    g = np.ascontiguousarray(g, dtype=np.float64)
    gg = np.zeros_like(g)
    lib().orc_ghost(C.byref(p), tag, _dp(W), _dp(g), _dp(n), _dp(Wg), _dp(gg))
    return Wg, gg


def coloring_graph(xadj, adj):
    n = len(xadj) - 1
    xadj = np.ascontiguousarray(xadj, dtype=np.int32)
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    col = np.zeros(n, dtype=np.int32)
    nc = C.c_int32()
    lib().orc_coloring_graph(n, _ip(xadj), _ip(adj), _ip(col), C.byref(nc))
    return col, nc.value


def freestream(mach, dim=2, gamma=1.4, aoa_deg=0.0):
    """Free-stream conservative state (rho=1, |u|=Ma, p=1/gamma)."""
    a = np.deg2rad(aoa_deg)
    u = np.array([mach * np.cos(a), mach * np.sin(a), 0.0])[:dim]
    p = 1.0 / gamma
    return np.concatenate([[1.0], u, [p / (gamma - 1.0) + 0.5 * u @ u]])
