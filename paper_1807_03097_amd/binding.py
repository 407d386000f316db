"""Python binding of the igaefie C ABI (include/igaefie.h).

Argument marshalling only: every step of the method runs in the HIP library
`libigaefie.so` built in this directory.  The functions `ige_*` mirror the C
entry points one to one; `Context`, `Geometry` and `Operator` are thin owners of
the handles.  Device vectors are torch tensors (complex128, contiguous, on the
context's device); host vectors are numpy arrays.  There is no fallback: if the
library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os
import sys
import weakref

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libigaefie.so")

IGE_OK, IGE_EINVAL, IGE_ENOMEM, IGE_ENOTCONV, IGE_EDEVICE = 0, -1, -2, -3, -4
IGE_HOST, IGE_DEVICE = 0, 1


class IgeError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"igaefie error {code}: {msg}")
        self.code = code


class ige_params(C.Structure):
    _fields_ = [("p", C.c_int), ("level", C.c_int), ("kappa", C.c_double), ("q", C.c_int), ("eta", C.c_double),
                ("gauss_near", C.c_int), ("gauss_singular", C.c_int), ("leaf_depth", C.c_int),
                ("store_coupling", C.c_int), ("kappa_cap", C.c_double), ("kind", C.c_int),
                ("q_level", C.c_int * 11)]


class ige_op_info_t(C.Structure):
    _fields_ = [("n_dof", C.c_int64), ("n_elements", C.c_int64), ("near_nnz", C.c_int64),
                ("far_pairs", C.c_int64), ("near_leaf_pairs", C.c_int64), ("singular_pairs", C.c_int64),
                ("leaf_level", C.c_int32), ("q", C.c_int32), ("device_bytes", C.c_int64),
                ("assemble_ms", C.c_double), ("near_distinct", C.c_int64), ("q_level", C.c_int32 * 11),
                ("level_diam", C.c_double * 11), ("m2l_unordered", C.c_int32)]


IGE_F64, IGE_F32, IGE_BF16, IGE_BF16X3, IGE_BF16X3_ALL = 0, 1, 2, 3, 4
IGE_OP_EFIE, IGE_OP_SCALAR = 0, 1
IGE_PROBE_HBM, IGE_PROBE_MFMA_BF16, IGE_PROBE_MFMA_F64 = 0, 1, 2
IGE_RHS_PLANE, IGE_RHS_POINT = 0, 1


class ige_solve_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("restart", C.c_int), ("maxit", C.c_int), ("refine", C.c_int),
                ("inner_tol", C.c_double), ("inner_prec", C.c_int)]


class ige_solve_stats(C.Structure):
    _fields_ = [("iters", C.c_int), ("outer", C.c_int), ("relres", C.c_double), ("seconds", C.c_double)]


class ige_srv_stats(C.Structure):
    _fields_ = [("state", C.c_int), ("rc", C.c_int), ("iters", C.c_int), ("relres", C.c_double),
                ("n_dof", C.c_int64), ("footprint", C.c_size_t), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double), ("assemble_s", C.c_double),
                ("solve_s", C.c_double), ("n_waves", C.c_int), ("merged", C.c_int), ("reused", C.c_int)]


# One HIP runtime per process: torch ships its own libamdhip64 (same soname);
# loading torch first lets this library bind to that runtime instead of a second one.
try:
    import torch  # noqa: F401
except ImportError:   # torch is optional for host-pointer use
    torch = None

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or paper_1807_03097_amd/build.py")
_lib = C.CDLL(LIB_PATH)

_V = C.c_void_p
_SIGS = {
    "ige_last_error": (C.c_char_p, []),
    "ige_version": (C.c_char_p, []),
    "ige_ctx_create": (C.c_int, [C.c_int, _V, C.POINTER(_V)]),
    "ige_ctx_destroy": (C.c_int, [_V]),
    "ige_geom_create": (C.c_int, [_V, C.c_int, _V, _V, _V, _V, C.POINTER(_V)]),
    "ige_geom_destroy": (C.c_int, [_V]),
    "ige_op_assemble": (C.c_int, [_V, C.POINTER(ige_params), C.POINTER(_V)]),
    "ige_op_plan": (C.c_int, [_V, C.POINTER(ige_params), C.POINTER(_V)]),
    "ige_op_destroy": (C.c_int, [_V]),
    "ige_op_info": (C.c_int, [_V, C.POINTER(ige_op_info_t)]),
    "ige_op_dofmap": (C.c_int, [_V, _V, _V]),
    "ige_op_partition": (C.c_int, [_V, _V, _V]),
    "ige_op_near_blocks": (C.c_int, [_V, _V, C.c_int64]),
    "ige_apply": (C.c_int, [_V, C.c_int, _V, _V, C.c_int]),
    "ige_apply_prec": (C.c_int, [_V, C.c_int, _V, _V, C.c_int, C.c_int]),
    "ige_op_set_profiling": (C.c_int, [_V, C.c_int]),
    "ige_op_set_overlap": (C.c_int, [_V, C.c_int]),
    "ige_op_stage_times": (C.c_int, [_V, _V, C.c_int]),
    "ige_op_autotune": (C.c_int, [_V, C.c_int, C.c_int, _V, C.c_int]),
    "ige_rhs_plane_wave": (C.c_int, [_V, C.c_int, _V, _V, _V, C.c_int]),
    "ige_rhs_scalar": (C.c_int, [_V, C.c_int, C.c_int, _V, _V, C.c_int]),
    "ige_solve": (C.c_int, [_V, C.c_int, _V, _V, C.c_int, C.POINTER(ige_solve_opts), _V]),
    "ige_helmholtz_eval": (C.c_int, [_V, C.c_int64, C.c_double, _V, _V, C.c_int]),
    "ige_peak_probe": (C.c_int, [_V, C.c_int, C.POINTER(C.c_double)]),
    "ige_potential": (C.c_int, [_V, C.c_int, _V, C.c_int, C.c_int, _V, _V]),
    "ige_potential_noalloc": (C.c_int, [_V, C.c_int, _V, C.c_int, _V, _V]),
    "ige_srv_create": (C.c_int, [_V, C.c_int, C.c_size_t, C.POINTER(_V)]),
    "ige_srv_submit": (C.c_int, [_V, _V, C.POINTER(ige_params), _V, _V, C.POINTER(ige_solve_opts),
                                 C.POINTER(C.c_int64)]),
    "ige_srv_submit_waves": (C.c_int, [_V, _V, C.POINTER(ige_params), C.c_int, _V, _V,
                                       C.POINTER(ige_solve_opts), C.POINTER(C.c_int64)]),
    "ige_srv_set_merge": (C.c_int, [_V, C.c_int]),
    "ige_srv_poll": (C.c_int, [_V, C.c_int64, C.POINTER(ige_srv_stats)]),
    "ige_srv_wait": (C.c_int, [_V, C.c_int64, C.POINTER(ige_srv_stats)]),
    "ige_srv_result": (C.c_int, [_V, C.c_int64, _V, C.c_int64]),
    "ige_srv_destroy": (C.c_int, [_V]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(rc):
    if rc < 0:
        raise IgeError(rc, _lib.ige_last_error().decode())
    return rc


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(_V)
    return _V(a.data_ptr())   # torch tensor


def _kind(a):
    return IGE_HOST if isinstance(a, np.ndarray) else IGE_DEVICE


# --- one-to-one wrappers -------------------------------------------------------
def ige_last_error():
    return _lib.ige_last_error().decode()


def ige_version():
    return _lib.ige_version().decode()


def ige_ctx_create(device=0, stream=None):
    h = _V()
    _check(_lib.ige_ctx_create(device, _V(stream) if stream else None, C.byref(h)))
    return h


def ige_ctx_destroy(h):
    _check(_lib.ige_ctx_destroy(h))


def ige_geom_create(ctx, deg, nctrl, knots, ctrl):
    deg = np.ascontiguousarray(deg, np.int32)
    nctrl = np.ascontiguousarray(nctrl, np.int32)
    knots = np.ascontiguousarray(knots, np.float64)
    ctrl = np.ascontiguousarray(ctrl, np.float64)
    h = _V()
    _check(_lib.ige_geom_create(ctx, len(deg) // 2, _ptr(deg), _ptr(nctrl), _ptr(knots), _ptr(ctrl), C.byref(h)))
    return h


def ige_geom_destroy(h):
    _check(_lib.ige_geom_destroy(h))


def ige_op_assemble(geom, prm: ige_params):
    h = _V()
    _check(_lib.ige_op_assemble(geom, C.byref(prm), C.byref(h)))
    return h


def ige_op_plan(geom, prm: ige_params):
    h = _V()
    _check(_lib.ige_op_plan(geom, C.byref(prm), C.byref(h)))
    return h


def ige_op_destroy(h):
    _check(_lib.ige_op_destroy(h))


def ige_op_info(op):
    info = ige_op_info_t()
    _check(_lib.ige_op_info(op, C.byref(info)))
    return info


def ige_op_dofmap(op, dof, sgn):
    _check(_lib.ige_op_dofmap(op, _ptr(dof), _ptr(sgn)))


def ige_op_partition(op, far, near):
    _check(_lib.ige_op_partition(op, _ptr(far), _ptr(near)))


def ige_apply(op, r, x, y, ptr_kind):
    _check(_lib.ige_apply(op, r, _ptr(x), _ptr(y), ptr_kind))


def ige_apply_prec(op, r, x, y, ptr_kind, prec):
    _check(_lib.ige_apply_prec(op, r, _ptr(x), _ptr(y), ptr_kind, prec))


def ige_op_set_profiling(op, on):
    _check(_lib.ige_op_set_profiling(op, int(on)))


def ige_op_set_overlap(op, on):
    _check(_lib.ige_op_set_overlap(op, int(on)))


def ige_op_stage_times(op):
    ms = np.zeros(9)
    n = _check(_lib.ige_op_stage_times(op, _ptr(ms), 9))
    return ms[:n]


def ige_rhs_plane_wave(op, r, dirs, pols, f, ptr_kind):
    dirs = np.ascontiguousarray(dirs, np.float64)
    pols = np.ascontiguousarray(pols, np.complex128)
    _check(_lib.ige_rhs_plane_wave(op, r, _ptr(dirs), _ptr(pols), _ptr(f), ptr_kind))


def ige_peak_probe(ctx, kind):
    """achievable device peak: GB/s (IGE_PROBE_HBM) or TFLOP/s (the matrix-core kinds)"""
    v = C.c_double(0.0)
    _check(_lib.ige_peak_probe(ctx, int(kind), C.byref(v)))
    return v.value


def ige_rhs_scalar(op, r, kind, a, f, ptr_kind):
    a = np.ascontiguousarray(a, np.float64)
    _check(_lib.ige_rhs_scalar(op, r, kind, _ptr(a), _ptr(f), ptr_kind))


def ige_solve(op, r, f, x, ptr_kind, opts: ige_solve_opts, stats=None):
    arr = (ige_solve_stats * r)() if stats is None else stats
    rc = _lib.ige_solve(op, r, _ptr(f), _ptr(x), ptr_kind, C.byref(opts), C.cast(arr, _V))
    if rc < 0 and rc != IGE_ENOTCONV:
        _check(rc)
    return rc, arr


def ige_helmholtz_eval(ctx, kappa, r2, prec=IGE_F64):
    r2 = np.ascontiguousarray(r2, np.float64)
    out = np.zeros(len(r2), np.complex128)
    _check(_lib.ige_helmholtz_eval(ctx, len(r2), kappa, _ptr(r2), _ptr(out), prec))
    return out


# --- owners ---------------------------------------------------------------------
class Context:
    """device=-1 creates a host-only context (planning only, no HIP calls)."""

    def __init__(self, device: int = 0, stream=None):
        self.device = device
        self.h = ige_ctx_create(device, stream)
        self._deps = weakref.WeakSet()   # geometries, operators and servers made on it

    def close(self):
        """Destroy the context; servers, operators and geometries still open on it are
        closed first (the library refuses to destroy a context that has any)."""
        if self.h:
            deps = list(self._deps)
            for kind in (Server, Operator, Geometry):
                for d in deps:
                    if isinstance(d, kind):
                        d.close()
            ige_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        if sys.is_finalizing():   # the HIP runtime may already be gone
            return
        try:
            self.close()
        except Exception:
            pass


class Geometry:
    def __init__(self, ctx: Context, patches):
        from . import workloads
        self.ctx = ctx
        self.h = ige_geom_create(ctx.h, *workloads.pack(patches))
        ctx._deps.add(self)

    def close(self):
        if self.h:
            ige_geom_destroy(self.h)
            self.h = None

    def __del__(self):
        if sys.is_finalizing():   # the HIP runtime may already be gone
            return
        try:
            self.close()
        except Exception:
            pass


def _levels(q_level):
    """ige_params.q_level from a sequence of per-level degrees (0: the base q)"""
    arr = (C.c_int * 11)()
    if q_level is not None:
        ql = [int(v) for v in q_level]
        if len(ql) > 11:
            raise ValueError("at most 11 levels")
        for i, v in enumerate(ql):
            arr[i] = v
    return arr


def degree_rule(info, kappa: float, q: int, far_levels, qmax: int = 15, extra: int = 5):
    """Interpolation degree per level that grows with the oscillation of the kernel
    over the level's clusters: q_l = min(qmax, max(q, ceil(kappa diam_l / 2) + extra))
    on the levels that have far blocks (far_levels), q elsewhere; diam_l from the
    operator info (ige_op_info of a planned operator)."""
    import math
    out = []
    for lvl in range(int(info.leaf_level) + 1):
        if lvl in far_levels:
            out.append(int(min(qmax, max(q, math.ceil(kappa * info.level_diam[lvl] / 2) + extra))))
        else:
            out.append(int(q))
    return out


class Operator:
    def __init__(self, geom: Geometry, p: int, level: int, kappa: float, q: int = 8, eta: float = 1.0,
                 gauss_near: int = 5, gauss_singular: int = 5, leaf_depth: int = -1, plan_only: bool = False,
                 store_coupling: int = -1, kappa_cap: float = 0.0, kind: int = IGE_OP_EFIE, q_level=None):
        self.geom = geom
        self.prm = ige_params(p, level, kappa, q, eta, gauss_near, gauss_singular, leaf_depth, store_coupling,
                              kappa_cap, kind, _levels(q_level))
        self.h = ige_op_plan(geom.h, self.prm) if plan_only else ige_op_assemble(geom.h, self.prm)
        geom.ctx._deps.add(self)
        self.info = ige_op_info(self.h)
        self.N = int(self.info.n_dof)
        self.p, self.level = p, level

    def close(self):
        if self.h:
            ige_op_destroy(self.h)
            self.h = None

    def __del__(self):
        if sys.is_finalizing():   # the HIP runtime may already be gone
            return
        try:
            self.close()
        except Exception:
            pass

    def dofmap(self):
        nb = (1 << self.level) + self.p
        P = self.geom_patches()
        dof = np.zeros((P, 2, nb, nb), np.int32)
        sgn = np.zeros((P, 2, nb, nb), np.int8)
        ige_op_dofmap(self.h, dof, sgn)
        return dof, sgn

    def geom_patches(self):
        return int(self.info.n_elements) >> (2 * self.level)

    def q_levels(self):
        """interpolation degree of each level 0..leaf level"""
        return [int(self.info.q_level[l]) for l in range(int(self.info.leaf_level) + 1)]

    def level_diameters(self):
        return [float(self.info.level_diam[l]) for l in range(int(self.info.leaf_level) + 1)]

    def partition(self):
        far = np.zeros((int(self.info.far_pairs), 3), np.int32)
        near = np.zeros((int(self.info.near_leaf_pairs), 2), np.int32)
        ige_op_partition(self.h, far, near)
        return {"L": int(self.info.leaf_level), "far": far, "near": near}

    def near_blocks(self):
        """the stored near-field blocks as a flat complex array of near_nnz entries"""
        out = np.zeros(int(self.info.near_nnz), np.complex128)
        _check(_lib.ige_op_near_blocks(self.h, _ptr(out), len(out)))
        return out

    def apply(self, x, y=None, prec=IGE_F64):
        """y = A x; x numpy (host) or torch (device) of shape (N,) or (r, N)."""
        r = 1 if x.ndim == 1 else x.shape[0]
        if y is None:
            if isinstance(x, np.ndarray):
                y = np.zeros_like(x, dtype=np.complex128)
            else:
                y = x.new_zeros(x.shape)
        ige_apply_prec(self.h, r, x, y, _kind(x), prec)
        return y

    def rhs_plane_wave(self, dirs, pols, out=None):
        dirs = np.atleast_2d(dirs)
        r = dirs.shape[0]
        if out is None:
            out = np.zeros((r, self.N), np.complex128)
        ige_rhs_plane_wave(self.h, r, dirs, np.atleast_2d(pols), out, _kind(out))
        return out

    def rhs_scalar(self, kind, a, out=None):
        """scalar single layer data moments: kind IGE_RHS_PLANE (a: directions) or
        IGE_RHS_POINT (a: source points), a of shape (3,) or (r, 3)"""
        a = np.atleast_2d(np.asarray(a, np.float64))
        r = a.shape[0]
        if out is None:
            out = np.zeros((r, self.N), np.complex128)
        ige_rhs_scalar(self.h, r, int(kind), a, out, _kind(out))
        return out

    def solve(self, f, x0=None, tol=1e-8, restart=1500, maxit=10000, refine=False, inner_tol=1e-4,
              inner_prec=IGE_F32):
        """GMRES (all right-hand sides at once); returns (x, [(iters, outer, relres, seconds)], rc)."""
        r = 1 if f.ndim == 1 else f.shape[0]
        if x0 is None:
            x0 = np.zeros_like(f) if isinstance(f, np.ndarray) else f.new_zeros(f.shape)
        opts = ige_solve_opts(tol, restart, maxit, int(refine), inner_tol, inner_prec)
        rc, stats = ige_solve(self.h, r, f, x0, _kind(f), opts)
        return x0, [(s.iters, s.outer, s.relres, s.seconds) for s in stats], rc

    def potential(self, w, points):
        """scattered field e_s = V~ w at points [npts][3] -> [npts][3] (or [r][npts][3])"""
        points = np.ascontiguousarray(points, np.float64).reshape(-1, 3)
        r = 1 if w.ndim == 1 else w.shape[0]
        out = np.zeros((r, len(points), 3), np.complex128)
        _check(_lib.ige_potential(self.h, r, _ptr(w), _kind(w), len(points), _ptr(points), _ptr(out)))
        return out[0] if w.ndim == 1 else out

    def potential_noalloc(self, w, points, out):
        """ige_potential_noalloc: w [N] or [r][N], points [npts][3] (float64) and out
        [npts][3] or [r][npts][3] (complex128), all torch tensors on the context's
        device; ordered on the context's stream"""
        r = 1 if w.ndim == 1 else w.shape[0]
        npts = points.shape[0]
        _check(_lib.ige_potential_noalloc(self.h, r, _ptr(w), npts, _ptr(points), _ptr(out)))
        return out

    def autotune(self, r, prec=IGE_F64):
        """time the candidate tile shapes of the r-column apply and keep the fastest;
        returns {knob: value} for the knobs that apply uses"""
        ch = np.full(7, -1, np.int32)
        _check(_lib.ige_op_autotune(self.h, int(r), int(prec), _ptr(ch), 7))
        names = ("m2l_ncol", "near_bx_nt", "near_mfma_nt", "m2l_rb", "m2l_double_buffer", "m2l_order",
                 "m2l_f64_matrix_cores")
        return {n: int(v) for n, v in zip(names, ch) if v >= 0}

    def set_profiling(self, on=True):
        """on: True/1 every stage boundary, 2 the block pass and coupling kernel only, False/0 off"""
        ige_op_set_profiling(self.h, int(on))

    def set_overlap(self, on=True):
        ige_op_set_overlap(self.h, on)

    def stage_times(self):
        return ige_op_stage_times(self.h)


# --- serving ---------------------------------------------------------------------
def ige_srv_create(ctx, n_workers=4, hbm_budget=0):
    h = _V()
    _check(_lib.ige_srv_create(ctx, n_workers, hbm_budget, C.byref(h)))
    return h


def ige_srv_submit(srv, geom, prm, direction, pol, opts):
    d = np.ascontiguousarray(direction, np.float64)
    pl = np.ascontiguousarray(pol, np.complex128)
    t = C.c_int64()
    _check(_lib.ige_srv_submit(srv, geom, C.byref(prm), _ptr(d), _ptr(pl), C.byref(opts), C.byref(t)))
    return t.value


def ige_srv_submit_waves(srv, geom, prm, directions, pols, opts):
    d = np.ascontiguousarray(directions, np.float64).reshape(-1, 3)
    pl = np.ascontiguousarray(pols, np.complex128).reshape(-1, 3)
    if len(d) != len(pl):
        raise ValueError("directions and polarisations differ in number")
    t = C.c_int64()
    _check(_lib.ige_srv_submit_waves(srv, geom, C.byref(prm), len(d), _ptr(d), _ptr(pl), C.byref(opts),
                                     C.byref(t)))
    return t.value


def ige_srv_poll(srv, ticket):
    st = ige_srv_stats()
    _check(_lib.ige_srv_poll(srv, ticket, C.byref(st)))
    return st


def ige_srv_wait(srv, ticket):
    st = ige_srv_stats()
    _check(_lib.ige_srv_wait(srv, ticket, C.byref(st)))
    return st


def ige_srv_result(srv, ticket, n):
    x = np.zeros(n, np.complex128)
    _check(_lib.ige_srv_result(srv, ticket, _ptr(x), n))
    return x


def ige_srv_destroy(srv):
    _check(_lib.ige_srv_destroy(srv))


def _stats_dict(st):
    return {k: getattr(st, k) for k, _ in ige_srv_stats._fields_}


class Server:
    """Queue of independent scattering solves on one device (see ige_srv_create)."""

    def __init__(self, ctx: Context, n_workers: int = 4, hbm_budget: int = 0, max_merge: int | None = None):
        self.ctx = ctx
        self.h = ige_srv_create(ctx.h, n_workers, hbm_budget)
        ctx._deps.add(self)
        self._geoms = {}
        if max_merge is not None:
            _check(_lib.ige_srv_set_merge(self.h, int(max_merge)))

    def submit(self, geom: Geometry, p, level, kappa, direction, pol, q=8, eta=1.0, leaf_depth=-1,
               gauss_near=5, gauss_singular=5, tol=1e-6, restart=1500, maxit=10000, refine=False,
               inner_tol=1e-4, inner_prec=IGE_F32, kappa_cap=0.0, kind=IGE_OP_EFIE, q_level=None):
        prm = ige_params(p, level, kappa, q, eta, gauss_near, gauss_singular, leaf_depth, 0, kappa_cap, kind,
                         _levels(q_level))
        opts = ige_solve_opts(tol, restart, maxit, int(refine), inner_tol, inner_prec)
        if np.ndim(direction) == 2:   # [W][3] directions and polarisations: one request of W waves
            t = ige_srv_submit_waves(self.h, geom.h, prm, direction, pol, opts)
        else:
            t = ige_srv_submit(self.h, geom.h, prm, direction, pol, opts)
        self._geoms[t] = geom   # keep the geometry alive until the request is done
        return t

    def poll(self, ticket):
        return _stats_dict(ige_srv_poll(self.h, ticket))

    def wait(self, ticket):
        return _stats_dict(ige_srv_wait(self.h, ticket))

    def result(self, ticket):
        """Solution [N] of a single-wave request submitted with one direction, else [W][N]."""
        st = self.wait(ticket)
        x = ige_srv_result(self.h, ticket, st["n_waves"] * st["n_dof"])
        return (x.reshape(st["n_waves"], st["n_dof"]) if st["n_waves"] > 1 else x), st

    def close(self):
        if self.h:
            ige_srv_destroy(self.h)
            self.h = None
            self._geoms.clear()

    def __del__(self):
        if sys.is_finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
