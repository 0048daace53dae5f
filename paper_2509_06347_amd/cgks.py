"""ctypes binding of libcgks (argument marshalling only; see include/cgks.h).

Function names follow the C ABI without the ``cgks_`` prefix on the
:class:`Solver` methods.  Arrays may be numpy arrays (host memory) or torch
tensors on the HIP device (device memory, passed as raw pointers).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libcgks.so")

if not os.path.exists(LIBPATH):
    raise ImportError(f"{LIBPATH} is missing: build it with __graft_entry__.build() "
                      "or python paper_2509_06347_amd/build.py (no CPU fallback exists)")

_lib = C.CDLL(LIBPATH)

OK, NOTCONV, EINVAL, EMESH, EDEVICE, ENONPHYS, ELIMIT = 0, 1, -1, -2, -3, -4, -5
HOST, DEVICE = 0, 1
FP64, MIXED = 0, 1
TAG_FARFIELD, TAG_SLIP, TAG_ISOTHERMAL, TAG_ADIABATIC = 1, 2, 3, 4


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


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_nodes", C.c_int), ("coords", C.POINTER(C.c_double)),
                ("n_cells", C.c_int), ("cell_nodes", C.POINTER(C.c_int32)),
                ("n_bfaces", C.c_int), ("bface_nodes", C.POINTER(C.c_int32)),
                ("bface_tag", C.POINTER(C.c_int32)),
                ("cell_offsets", C.POINTER(C.c_int32)), ("bface_offsets", C.POINTER(C.c_int32))]


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I = C.POINTER(C.c_int32)
_sigs = {
    "cgks_default_params": (None, [C.POINTER(Params)]),
    "cgks_create": (C.c_int, [C.POINTER(Params), C.POINTER(_P)]),
    "cgks_destroy": (None, [_P]),
    "cgks_last_error": (C.c_char_p, [_P]),
    "cgks_strerror": (C.c_char_p, [C.c_int]),
    "cgks_set_stream": (C.c_int, [_P, _P]),
    "cgks_mesh_setup": (C.c_int, [_P, C.POINTER(Mesh), C.c_int, C.POINTER(_I)]),
    "cgks_level_size": (C.c_int, [_P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "cgks_coloring": (C.c_int, [_P, C.c_int, _I, _I]),
    "cgks_agglomerate": (C.c_int, [_P, C.c_int, _I, _I]),
    "cgks_cell_geometry": (C.c_int, [_P, C.c_int, _D, _D]),
    "cgks_init_freestream": (C.c_int, [_P]),
    "cgks_set_state": (C.c_int, [_P, _P, _P, _P, C.c_int]),
    "cgks_get_state": (C.c_int, [_P, _P, _P, _P, C.c_int]),
    "cgks_set_level_state": (C.c_int, [_P, C.c_int, _P, _P, _P, _P]),
    "cgks_get_level_state": (C.c_int, [_P, C.c_int, _P, _P, _P, _P]),
    "cgks_residual": (C.c_int, [_P, C.c_int, _P, _P, _P, C.c_int]),
    "cgks_time_steps": (C.c_int, [_P, C.c_int, _P, _P]),
    "cgks_smooth": (C.c_int, [_P, C.c_int, C.c_int]),
    "cgks_restrict": (C.c_int, [_P, C.c_int]),
    "cgks_prolong": (C.c_int, [_P, C.c_int]),
    "cgks_vcycle": (C.c_int, [_P, _D]),
    "cgks_solve": (C.c_int, [_P, C.c_double, C.c_int, C.POINTER(C.c_int), _D, C.c_int]),
    "cgks_run_cycles": (C.c_int, [_P, C.c_int, _D]),
    "cgks_stats": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "cgks_time_kernel": (C.c_int, [_P, C.c_int, C.c_int, _D, C.POINTER(C.c_int64)]),
    "cgks_autotune": (C.c_int, [_P]),
    "cgks_launch_shapes": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "cgks_coarse_shapes": (C.c_int, [_P, C.POINTER(C.c_int), C.c_int]),
    "cgks_set_coarse_shapes": (C.c_int, [_P, C.POINTER(C.c_int), C.c_int]),
    "cgks_batch_create": (C.c_int, [C.c_int, C.POINTER(_P), C.POINTER(_P)]),
    "cgks_batch_autotune": (C.c_int, [_P]),
    "cgks_batch_run_cycles": (C.c_int, [_P, C.c_int, _D]),
    "cgks_batch_solve": (C.c_int, [_P, C.c_double, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "cgks_batch_get_state": (C.c_int, [_P]),
    "cgks_batch_destroy": (None, [_P]),
    "cgks_mlp_create": (C.c_int, [C.POINTER(_P), C.c_int]),
    "cgks_mlp_destroy": (None, [_P]),
    "cgks_mlp_set_stream": (C.c_int, [_P, _P]),
    "cgks_mlp_num_params": (C.c_int, []),
    "cgks_mlp_get_weights": (C.c_int, [_P, _P]),
    "cgks_mlp_set_weights": (C.c_int, [_P, _P]),
    "cgks_mlp_forward": (C.c_int, [_P, _P, _P, C.c_int]),
    "cgks_mlp_forward_noalloc": (C.c_int, [_P, _P, _P, C.c_int]),
    "cgks_mlp_grads": (C.c_int, [_P, _P, _P, C.c_int, _P, C.POINTER(C.c_float)]),
    "cgks_mlp_train_step": (C.c_int, [_P, _P, _P, C.c_int, C.c_float, C.POINTER(C.c_float)]),
    "cgks_init_from_mlp": (C.c_int, [_P, _P, _P, _P, _P, _P, C.POINTER(C.c_int)]),
    "cgks_mlp_set_range": (C.c_int, [_P, _P, _P]),
    "cgks_mlp_features": (C.c_int, [_P, _P, C.c_int]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTS = tuple(_sigs)


class CgksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_lib.cgks_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def default_params(**kw):
    p = Params()
    _lib.cgks_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def _ptr(a):
    """Raw pointer and memory kind of a numpy array or a device tensor (None -> NULL)."""
    if a is None:
        return None, HOST
    if isinstance(a, np.ndarray):
        return a.ctypes.data, HOST
    if hasattr(a, "data_ptr"):
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return a.data_ptr(), (DEVICE if a.is_cuda else HOST)
    raise TypeError(type(a))


class Solver:
    """One solver context on one mesh (see include/cgks.h)."""

    def __init__(self, mesh, n_levels=3, use_parents=True, stream=None, **params):
        params.setdefault("dim", mesh.dim)
        params.setdefault("n_levels", n_levels)
        self.params = default_params(**params)
        self.dim = mesh.dim
        self.nvar = mesh.dim + 2
        ctx = _P()
        rc = _lib.cgks_create(C.byref(self.params), C.byref(ctx))
        if rc != OK:
            raise CgksError(rc, "cgks_create")
        self.ctx = ctx
        if stream is not None:
            self._check(_lib.cgks_set_stream(self.ctx, _P(stream)))
        keep = [np.ascontiguousarray(mesh.coords, dtype=np.float64),
                np.ascontiguousarray(mesh.cells, dtype=np.int32),
                np.ascontiguousarray(mesh.bfaces, dtype=np.int32),
                np.ascontiguousarray(mesh.btags, dtype=np.int32)]
        m = Mesh(mesh.dim, mesh.n_nodes, keep[0].ctypes.data_as(_D), mesh.n_cells,
                 keep[1].ctypes.data_as(_I), len(keep[3]), keep[2].ctypes.data_as(_I),
                 keep[3].ctypes.data_as(_I))
        if getattr(mesh, "cell_offsets", None) is not None:   # hybrid elements
            keep += [np.ascontiguousarray(mesh.cell_offsets, dtype=np.int32),
                     np.ascontiguousarray(mesh.bface_offsets, dtype=np.int32)]
            m.cell_offsets, m.bface_offsets = keep[4].ctypes.data_as(_I), keep[5].ctypes.data_as(_I)
        par = (_I * max(n_levels - 1, 1))()
        for l in range(n_levels - 1):
            if use_parents and l < len(mesh.parents):
                a = np.ascontiguousarray(mesh.parents[l], dtype=np.int32)
                keep.append(a)
                par[l] = a.ctypes.data_as(_I)
            else:
                par[l] = _I()
        self._check(_lib.cgks_mesh_setup(self.ctx, C.byref(m), n_levels, par))
        self.n_levels = n_levels
        self.sizes = []
        for l in range(n_levels):
            nc, nf = C.c_int(), C.c_int()
            self._check(_lib.cgks_level_size(self.ctx, l, C.byref(nc), C.byref(nf)))
            self.sizes.append((nc.value, nf.value))

    def _check(self, rc):
        if rc < 0:
            raise CgksError(rc, _lib.cgks_last_error(self.ctx).decode())
        return rc

    def close(self):
        if getattr(self, "ctx", None):
            _lib.cgks_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # set-up queries ----------------------------------------------------------
    def coloring(self, level):
        n = self.sizes[level][0]
        col = np.zeros(n, dtype=np.int32)
        nc = C.c_int32()
        self._check(_lib.cgks_coloring(self.ctx, level, col.ctypes.data_as(_I), C.byref(nc)))
        return col, nc.value

    def agglomerate(self, level=0):
        n = self.sizes[level][0]
        agg = np.zeros(n, dtype=np.int32)
        nc = C.c_int32()
        self._check(_lib.cgks_agglomerate(self.ctx, level, agg.ctypes.data_as(_I), C.byref(nc)))
        return agg, nc.value

    def cell_geometry(self, level=0):
        n = self.sizes[level][0]
        V, Cc = np.zeros(n), np.zeros((n, self.dim))
        self._check(_lib.cgks_cell_geometry(self.ctx, level, V.ctypes.data_as(_D), Cc.ctypes.data_as(_D)))
        return V, Cc

    def mlp_features(self):
        """Raw warm-start features [n, 5] (float32) of the fine cells: Mach,
        log10 Re, centroid x, y, distance to the nearest wall-face centre."""
        X = np.zeros((self.sizes[0][0], 5), dtype=np.float32)
        self._check(_lib.cgks_mlp_features(self.ctx, X.ctypes.data, HOST))
        return X

    # state -------------------------------------------------------------------
    def init_freestream(self):
        self._check(_lib.cgks_init_freestream(self.ctx))

    def set_state(self, W, grad=None, alpha=None):
        arrs = [W, grad, alpha]
        if isinstance(W, np.ndarray):
            arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64) for a in arrs]
        ptrs = [_ptr(a) for a in arrs]
        mem = ptrs[0][1]
        self._check(_lib.cgks_set_state(self.ctx, ptrs[0][0], ptrs[1][0], ptrs[2][0], mem))

    def get_state(self):
        n = self.sizes[0][0]
        W = np.zeros((n, self.nvar))
        g = np.zeros((n, self.nvar, self.dim))
        a = np.zeros(n)
        self._check(_lib.cgks_get_state(self.ctx, W.ctypes.data, g.ctypes.data, a.ctypes.data, HOST))
        return W, g, a

    def get_state_into(self, W, grad=None, alpha=None):
        """Write the fine state into caller-provided arrays / device tensors."""
        p = [_ptr(x) for x in (W, grad, alpha)]
        self._check(_lib.cgks_get_state(self.ctx, p[0][0], p[1][0], p[2][0], p[0][1]))

    def set_level_state(self, level, W=None, W0=None, F=None, alpha=None):
        arrs = [None if x is None else np.ascontiguousarray(x, dtype=np.float64) for x in (W, W0, F, alpha)]
        self._check(_lib.cgks_set_level_state(self.ctx, level, *[None if a is None else a.ctypes.data for a in arrs]))

    def get_level_state(self, level):
        n = self.sizes[level][0]
        W, W0, F = (np.zeros((n, self.nvar)) for _ in range(3))
        a = np.zeros(n)
        self._check(_lib.cgks_get_level_state(self.ctx, level, W.ctypes.data, W0.ctypes.data,
                                              F.ctypes.data, a.ctypes.data))
        return W, W0, F, a

    # solver ------------------------------------------------------------------
    def residual(self, level=0):
        n = self.sizes[level][0]
        R = np.zeros((n, self.nvar))
        g = np.zeros((n, self.nvar, self.dim))
        a = np.zeros(n)
        self._check(_lib.cgks_residual(self.ctx, level, R.ctypes.data, g.ctypes.data, a.ctypes.data, HOST))
        return R, g, a

    def time_steps(self, level=0):
        n = self.sizes[level][0]
        de, di = np.zeros(n), np.zeros(n)
        self._check(_lib.cgks_time_steps(self.ctx, level, de.ctypes.data, di.ctypes.data))
        return de, di

    def smooth(self, level, n):
        self._check(_lib.cgks_smooth(self.ctx, level, n))

    def restrict(self, level):
        self._check(_lib.cgks_restrict(self.ctx, level))

    def prolong(self, level):
        self._check(_lib.cgks_prolong(self.ctx, level))

    def vcycle(self):
        nrm = C.c_double()
        self._check(_lib.cgks_vcycle(self.ctx, C.byref(nrm)))
        return nrm.value

    def run_cycles(self, n):
        hist = np.zeros(n)
        self._check(_lib.cgks_run_cycles(self.ctx, n, hist.ctypes.data_as(_D)))
        return hist

    def solve(self, tol=1e-10, max_cycles=1000):
        hist = np.zeros(max_cycles)
        ncyc = C.c_int()
        rc = self._check(_lib.cgks_solve(self.ctx, C.c_double(tol), max_cycles, C.byref(ncyc),
                                         hist.ctypes.data_as(_D), max_cycles))
        return rc, hist[:ncyc.value]

    def time_kernel(self, kernel, reps=20):
        """(average ms, work items) of fine-residual kernel 0/1/2 (recon/flux/gather)."""
        ms, n = C.c_double(), C.c_int64()
        self._check(_lib.cgks_time_kernel(self.ctx, kernel, reps, C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def autotune(self):
        self._check(_lib.cgks_autotune(self.ctx))
        return self.launch_shapes()

    def launch_shapes(self):
        r, f, g = C.c_int(), C.c_int(), C.c_int()
        self._check(_lib.cgks_launch_shapes(self.ctx, C.byref(r), C.byref(f), C.byref(g)))
        return r.value, f.value, g.value

    def coarse_shapes(self):
        """Cells per block of each coarse level's slot-parallel kernels (0: per-cell kernels)."""
        n = len(self.sizes) - 1
        a = (C.c_int * max(n, 1))()
        self._check(_lib.cgks_coarse_shapes(self.ctx, a, n))
        return [a[i] for i in range(n)]

    def set_coarse_shapes(self, cells_per_block):
        v = list(cells_per_block)
        a = (C.c_int * max(len(v), 1))(*v)
        self._check(_lib.cgks_set_coarse_shapes(self.ctx, a, len(v)))

    def stats(self):
        a, b = C.c_int64(), C.c_int64()
        self._check(_lib.cgks_stats(self.ctx, C.byref(a), C.byref(b)))
        return a.value, b.value


class Batch:
    """Independent problems advanced together (see cgks_batch_* in include/cgks.h)."""

    def __init__(self, solvers):
        self.solvers = list(solvers)
        arr = (_P * len(self.solvers))(*[s.ctx for s in self.solvers])
        h = _P()
        rc = _lib.cgks_batch_create(len(self.solvers), arr, C.byref(h))
        if rc != OK:
            raise CgksError(rc, "cgks_batch_create")
        self.h = h

    def _check(self, rc):
        if rc < 0:
            raise CgksError(rc, "batch")
        return rc

    def autotune(self):
        self._check(_lib.cgks_batch_autotune(self.h))

    def run_cycles(self, n):
        hist = np.zeros((len(self.solvers), n))
        self._check(_lib.cgks_batch_run_cycles(self.h, n, hist.ctypes.data_as(_D)))
        return hist

    def solve(self, tol=1e-10, max_cycles=1000):
        m = len(self.solvers)
        cyc = (C.c_int * m)()
        st = (C.c_int * m)()
        rc = _lib.cgks_batch_solve(self.h, C.c_double(tol), max_cycles, cyc, st)
        if rc < 0 and rc != ENONPHYS:
            raise CgksError(rc, "cgks_batch_solve")
        return rc, np.array(cyc[:]), np.array(st[:])

    def sync_states(self):
        self._check(_lib.cgks_batch_get_state(self.h))

    def close(self):
        if getattr(self, "h", None):
            _lib.cgks_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _f32(a, n):
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.size != n:
        raise ValueError(f"expected {n} values, got {a.size}")
    return a


class MLP:
    """Warm-start surrogate (see cgks_mlp_* in include/cgks.h).  X and Y are
    float32 device tensors of shape [n, 5] and [n, 4]."""

    SIZES = (5, 256, 256, 256, 4)
    NOALLOC_MAX_ROWS = 16384

    def __init__(self, seed=0, stream=None):
        h = _P()
        rc = _lib.cgks_mlp_create(C.byref(h), seed)
        if rc != OK:
            raise CgksError(rc, "cgks_mlp_create")
        self.h = h
        if stream is not None:
            self._check(_lib.cgks_mlp_set_stream(self.h, _P(stream)))

    @staticmethod
    def num_params():
        return _lib.cgks_mlp_num_params()

    def _check(self, rc, what="mlp"):
        if rc != OK:
            raise CgksError(rc, what)

    @staticmethod
    def _dev(t, cols):
        if not (hasattr(t, "is_cuda") and t.is_cuda) or str(t.dtype) != "torch.float32" or not t.is_contiguous():
            raise TypeError("expected a contiguous float32 device tensor")
        if t.dim() != 2 or t.shape[1] != cols:
            raise ValueError(f"expected shape [n, {cols}]")
        return t.data_ptr(), t.shape[0]

    def get_weights(self):
        w = np.zeros(self.num_params(), dtype=np.float32)
        self._check(_lib.cgks_mlp_get_weights(self.h, w.ctypes.data))
        return w

    def set_weights(self, flat):
        w = _f32(flat, self.num_params())
        self._check(_lib.cgks_mlp_set_weights(self.h, w.ctypes.data))

    def forward(self, X, Y):
        px, n = self._dev(X, 5)
        py, ny = self._dev(Y, 4)
        if ny != n:
            raise ValueError("X and Y differ in rows")
        self._check(_lib.cgks_mlp_forward(self.h, px, py, n), "cgks_mlp_forward")

    def forward_noalloc(self, X, Y):
        """cgks_mlp_forward_noalloc: the forward pass in the library's fixed
        workspace (at most NOALLOC_MAX_ROWS rows; calls on one device must not
        overlap)."""
        px, n = self._dev(X, 5)
        py, ny = self._dev(Y, 4)
        if ny != n:
            raise ValueError("X and Y differ in rows")
        self._check(_lib.cgks_mlp_forward_noalloc(self.h, px, py, n), "cgks_mlp_forward_noalloc")

    def grads(self, X, Y):
        px, n = self._dev(X, 5)
        py, _ = self._dev(Y, 4)
        g = np.zeros(self.num_params(), dtype=np.float32)
        loss = C.c_float()
        self._check(_lib.cgks_mlp_grads(self.h, px, py, n, g.ctypes.data, C.byref(loss)), "cgks_mlp_grads")
        return float(loss.value), g

    def train_step(self, X, Y, lr):
        px, n = self._dev(X, 5)
        py, _ = self._dev(Y, 4)
        loss = C.c_float()
        self._check(_lib.cgks_mlp_train_step(self.h, px, py, n, C.c_float(lr), C.byref(loss)), "cgks_mlp_train_step")
        return float(loss.value)

    def set_range(self, lo, hi):
        """Training range of the raw features; a warm start falls back to the
        free stream in cells outside it (None, None clears it)."""
        if lo is None:
            self._check(_lib.cgks_mlp_set_range(self.h, None, None))
            return
        a, b = _f32(lo, 5), _f32(hi, 5)
        self._check(_lib.cgks_mlp_set_range(self.h, a.ctypes.data, b.ctypes.data), "cgks_mlp_set_range")

    def init_solver(self, solver, fmean, fstd, tmean, tstd):
        """Warm-start a 2-D solver's fine state; returns the number of fallback cells."""
        fm, fs, tm, ts = _f32(fmean, 5), _f32(fstd, 5), _f32(tmean, 4), _f32(tstd, 4)
        nfb = C.c_int()
        rc = _lib.cgks_init_from_mlp(solver.ctx, self.h, fm.ctypes.data, fs.ctypes.data, tm.ctypes.data,
                                     ts.ctypes.data, C.byref(nfb))
        if rc != OK:
            raise CgksError(rc, _lib.cgks_last_error(solver.ctx).decode())
        return int(nfb.value)

    def close(self):
        if getattr(self, "h", None):
            _lib.cgks_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
