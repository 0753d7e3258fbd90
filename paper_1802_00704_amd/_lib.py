"""ctypes binding of libgks (include/gks.h): argument marshalling only.

Every computation runs in the HIP library; this module converts Python
objects to the C structures and torch tensors to device pointers.  It raises
if the library is missing or fails to load: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgks.so")

GKS_OK, GKS_EINVAL, GKS_ENOMEM, GKS_EHIP, GKS_ENOCONV, GKS_ENONPHYS = 0, -1, -2, -3, -4, -5
LIMIT_CONSERVATIVE, LIMIT_CHARACTERISTIC = 1, 2
GKS_FP64, GKS_MIXED = 0, 1
GKS_INNER_RICHARDSON, GKS_INNER_GMRES = 0, 1
GKS_ORDER_MULTICOLOR, GKS_ORDER_RCM = 0, 1

EXPORTS = ("gks_params_default", "gks_mesh_create", "gks_cls_reconstruct", "gks_flux", "gks_step",
           "gks_faces", "gks_mesh_get_stats", "gks_profile_enable", "gks_profile_get", "gks_apply_precond", "gks_limit",
           "gks_limit_noalloc", "gks_batch_create", "gks_batch_step", "gks_batch_last_error",
           "gks_batch_destroy",
           "gks_host_inspect", "gks_host_free", "gks_last_error", "gks_destroy")


class GksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


class NonConvergence(GksError):
    pass


class NonPhysical(GksError):
    pass


class MeshDesc(C.Structure):
    _fields_ = [("nv", C.c_int32), ("nt", C.c_int32), ("xy", C.POINTER(C.c_double)),
                ("tri", C.POINTER(C.c_int32)), ("edge_tag", C.POINTER(C.c_int32)),
                ("periodic_x", C.c_int32), ("periodic_y", C.c_int32), ("Lx", C.c_double), ("Ly", C.c_double),
                ("n_bc", C.c_int32), ("bc_kind", C.POINTER(C.c_int32)), ("bc_state", C.POINTER(C.c_double))]


class Params(C.Structure):
    _fields_ = [("gamma", C.c_double), ("mu", C.c_double), ("tau_eps", C.c_double), ("cls_w", C.c_double),
                ("cfl", C.c_double), ("tol", C.c_double), ("restart", C.c_int32), ("max_iter", C.c_int32),
                ("precision", C.c_int32), ("ordering", C.c_int32), ("inner_iters", C.c_int32),
                ("exact_time", C.c_int32), ("nonphys_fallback", C.c_int32), ("all_quadratic", C.c_int32),
                ("graphs", C.c_int32), ("graph_budget", C.c_int32), ("limiter", C.c_int32),
                ("reorth_tol", C.c_double), ("inner_solver", C.c_int32), ("inner_iters_first", C.c_int32),
                ("adapt_sweeps", C.c_int32), ("extrap_points", C.c_int32)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32 * 4), ("restarts", C.c_int32 * 4), ("rel_resid", C.c_double * 4),
                ("nonphys", C.c_int32), ("solve_ms", C.c_double), ("call_ms", C.c_double),
                ("limited", C.c_int32), ("reorth", C.c_int32),
                ("first_sweeps", C.c_int32), ("start_resid", C.c_double),
                ("start_points", C.c_int32)]

    def as_dict(self):
        return {"iters": list(self.iters), "restarts": list(self.restarts),
                "rel_resid": list(self.rel_resid), "nonphys": int(self.nonphys),
                "solve_ms": float(self.solve_ms), "call_ms": float(self.call_ms), "limited": int(self.limited),
                "reorth": int(self.reorth), "first_sweeps": int(self.first_sweeps),
                "start_resid": float(self.start_resid), "start_points": int(self.start_points)}


class Stats(C.Structure):
    _fields_ = [("nt", C.c_int32), ("nf", C.c_int32), ("nf_boundary", C.c_int32), ("n_levels", C.c_int32),
                ("n_colors", C.c_int32), ("rcm_bandwidth", C.c_int32), ("device_bytes", C.c_int64),
                ("graph_steps", C.c_int64), ("capture_failures", C.c_int32), ("split_form", C.c_int32),
                ("graph_captures", C.c_int32), ("capture_ms", C.c_double)]


class HostSystem(C.Structure):
    _fields_ = [("nt", C.c_int32), ("nf", C.c_int32), ("n_levels", C.c_int32), ("n_colors", C.c_int32),
                ("rcm_bandwidth", C.c_int32)] + [
        (name, C.POINTER(ctype)) for name, ctype in (
            ("own", C.c_int32), ("nbr", C.c_int32), ("area", C.c_double), ("h", C.c_double),
            ("perm", C.c_int32), ("lev_ptr", C.c_int32), ("kcol", C.c_int32), ("kval", C.c_double),
            ("lcol", C.c_int32), ("lval", C.c_double), ("ucol", C.c_int32), ("uval", C.c_double),
            ("dinv", C.c_double), ("spmv_order", C.c_int32))] + [("n_spmv_waves", C.c_int32)]


_lib = None


def lib():
    """Load libgks.so (raises OSError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError("libgks.so is not built: run `python -m paper_1802_00704_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.gks_params_default.argtypes = [C.POINTER(Params)]
        L.gks_params_default.restype = None
        L.gks_mesh_create.argtypes = [C.POINTER(MeshDesc), C.POINTER(Params), vp, C.POINTER(vp)]
        L.gks_mesh_create.restype = C.c_int
        L.gks_cls_reconstruct.argtypes = [vp, vp, vp, C.POINTER(SolveInfo)]
        L.gks_cls_reconstruct.restype = C.c_int
        L.gks_flux.argtypes = [vp, vp, vp, C.c_double, vp]
        L.gks_flux.restype = C.c_int
        L.gks_step.argtypes = [vp, vp, C.c_double, C.POINTER(C.c_double), C.POINTER(SolveInfo)]
        L.gks_step.restype = C.c_int
        L.gks_faces.argtypes = [vp, vp, vp]
        L.gks_limit.argtypes = [vp, vp, vp, vp, C.c_double, C.c_int32, C.POINTER(C.c_int32)]
        L.gks_limit.restype = C.c_int
        L.gks_limit_noalloc.argtypes = [vp, vp, vp, vp, C.c_double, C.c_int32, C.POINTER(C.c_int32)]
        L.gks_limit_noalloc.restype = C.c_int
        L.gks_apply_precond.argtypes = [vp, vp, vp, C.c_int]
        L.gks_apply_precond.restype = C.c_int
        L.gks_faces.restype = C.c_int
        L.gks_mesh_get_stats.argtypes = [vp, C.POINTER(Stats)]
        L.gks_mesh_get_stats.restype = C.c_int
        L.gks_profile_enable.argtypes = [vp, C.c_int]
        L.gks_profile_enable.restype = C.c_int
        L.gks_profile_get.argtypes = [vp, C.c_int, C.POINTER(C.c_char_p), C.POINTER(C.c_int64),
                                      C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.gks_profile_get.restype = C.c_int
        L.gks_host_inspect.argtypes = [C.POINTER(MeshDesc), C.POINTER(Params), C.POINTER(HostSystem)]
        L.gks_host_inspect.restype = C.c_int
        L.gks_host_free.argtypes = [C.POINTER(HostSystem)]
        L.gks_host_free.restype = None
        L.gks_last_error.argtypes = [vp]
        L.gks_last_error.restype = C.c_char_p
        L.gks_destroy.argtypes = [vp]
        L.gks_destroy.restype = None
        L.gks_batch_create.argtypes = [vp, C.POINTER(vp)]
        L.gks_batch_create.restype = C.c_int
        L.gks_batch_step.argtypes = [vp, C.c_int32, C.POINTER(vp), C.POINTER(vp), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double), C.POINTER(SolveInfo), C.POINTER(C.c_int32)]
        L.gks_batch_step.restype = C.c_int
        L.gks_batch_last_error.argtypes = [vp]
        L.gks_batch_last_error.restype = C.c_char_p
        L.gks_batch_destroy.argtypes = [vp]
        L.gks_batch_destroy.restype = None
        _lib = L
    return _lib


def default_params(**kw) -> Params:
    p = Params()
    lib().gks_params_default(C.byref(p))
    for key, val in kw.items():
        if not hasattr(p, key):
            raise KeyError("unknown parameter %r" % key)
        setattr(p, key, val)
    return p


def _check(code, handle=None):
    if code == GKS_OK:
        return
    msg = lib().gks_last_error(handle).decode(errors="replace")
    if code == GKS_ENOCONV:
        raise NonConvergence(code, msg)
    if code == GKS_ENONPHYS:
        raise NonPhysical(code, msg)
    raise GksError(code, msg)


def _dev(t, shape, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
        raise TypeError("%s must be a float64 CUDA tensor" % name)
    if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError("%s must be contiguous with shape %s, got %s" % (name, shape, tuple(t.shape)))
    return C.c_void_p(t.data_ptr())


def mesh_desc(mesh):
    """(MeshDesc, arrays kept alive) for a gks_inputs.Mesh-like object."""
    xy = np.ascontiguousarray(mesh.xy, dtype=np.float64)
    tri = np.ascontiguousarray(mesh.tri, dtype=np.int32)
    tag = np.ascontiguousarray(mesh.edge_tag, dtype=np.int32)
    kinds = np.array([k for k, _ in mesh.bc_table] or [0], dtype=np.int32)
    states = np.array([(s if s is not None else (0.0, 0.0, 0.0, 0.0)) for _, s in mesh.bc_table]
                      or [(0.0, 0.0, 0.0, 0.0)], dtype=np.float64).reshape(-1, 4)
    d = MeshDesc()
    d.nv = xy.shape[0]
    d.nt = tri.shape[0]
    d.xy = xy.ctypes.data_as(C.POINTER(C.c_double))
    d.tri = tri.ctypes.data_as(C.POINTER(C.c_int32))
    d.edge_tag = tag.ctypes.data_as(C.POINTER(C.c_int32))
    d.periodic_x = int(bool(mesh.periodic[0]))
    d.periodic_y = int(bool(mesh.periodic[1]))
    d.Lx, d.Ly = float(mesh.L[0]), float(mesh.L[1])
    d.n_bc = len(mesh.bc_table)
    d.bc_kind = kinds.ctypes.data_as(C.POINTER(C.c_int32))
    d.bc_state = states.ctypes.data_as(C.POINTER(C.c_double))
    return d, (xy, tri, tag, kinds, states)


def host_inspect(mesh, params: Params | None = None, **kw) -> dict:
    """Host-only per-mesh state (gks_host_inspect) as NumPy arrays."""
    prm = params if params is not None else default_params(**kw)
    d, keep = mesh_desc(mesh)
    hs = HostSystem()
    _check(lib().gks_host_inspect(C.byref(d), C.byref(prm), C.byref(hs)), None)
    try:
        nt, nf, nl = hs.nt, hs.nf, hs.n_levels
        arr = lambda ptr, n: np.ctypeslib.as_array(ptr, shape=(n,)).copy()
        out = {"nt": nt, "nf": nf, "n_levels": nl, "n_colors": hs.n_colors, "rcm_bandwidth": hs.rcm_bandwidth,
               "own": arr(hs.own, nf), "nbr": arr(hs.nbr, nf), "area": arr(hs.area, nt), "h": arr(hs.h, nt),
               "perm": arr(hs.perm, nt), "lev_ptr": arr(hs.lev_ptr, nl + 1),
               "kcol": arr(hs.kcol, 4 * nt).reshape(4, nt), "kval": arr(hs.kval, 100 * nt).reshape(4, 25, nt),
               "lcol": arr(hs.lcol, 3 * nt).reshape(3, nt), "lval": arr(hs.lval, 75 * nt).reshape(3, 25, nt),
               "ucol": arr(hs.ucol, 3 * nt).reshape(3, nt), "uval": arr(hs.uval, 75 * nt).reshape(3, 25, nt),
               "dinv": arr(hs.dinv, 25 * nt).reshape(25, nt),
               "spmv_order": arr(hs.spmv_order, hs.n_spmv_waves) if hs.n_spmv_waves else None}
    finally:
        lib().gks_host_free(C.byref(hs))
    return out


class GksMesh:
    """One mesh handle (gks_mesh) on the current HIP device."""

    def __init__(self, mesh, params: Params | None = None, stream=None, **kw):
        self._h = None
        prm = params if params is not None else default_params(**kw)
        d, self._keep = mesh_desc(mesh)
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        self.stream = stream
        sp = C.c_void_p(int(getattr(stream, "cuda_stream", stream) or 0))
        h = C.c_void_p()
        code = lib().gks_mesh_create(C.byref(d), C.byref(prm), sp, C.byref(h))
        _check(code, None)
        self._h = h
        self.params = prm
        st = self.stats()
        self.nt, self.nf = st["nt"], st["nf"]

    def close(self):
        if self._h is not None:
            lib().gks_destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def stats(self) -> dict:
        s = Stats()
        _check(lib().gks_mesh_get_stats(self._h, C.byref(s)), self._h)
        return {f: getattr(s, f) for f, _ in Stats._fields_}

    def faces(self):
        own = np.empty(self.nf, dtype=np.int32)
        nbr = np.empty(self.nf, dtype=np.int32)
        _check(lib().gks_faces(self._h, own.ctypes.data_as(C.c_void_p), nbr.ctypes.data_as(C.c_void_p)), self._h)
        return own, nbr

    def reconstruct(self, W, X=None):
        import torch
        if X is None:
            X = torch.empty((4, 5, self.nt), dtype=torch.float64, device=W.device)
        info = SolveInfo()
        code = lib().gks_cls_reconstruct(self._h, _dev(W, (4, self.nt), "W"), _dev(X, (4, 5, self.nt), "X"),
                                         C.byref(info))
        _check(code, self._h)
        return X, info.as_dict()

    def flux(self, W, X, dt, F=None):
        import torch
        if F is None:
            F = torch.empty((4, self.nf), dtype=torch.float64, device=W.device)
        code = lib().gks_flux(self._h, _dev(W, (4, self.nt), "W"), _dev(X, (4, 5, self.nt), "X"), float(dt),
                              _dev(F, (4, self.nf), "F"))
        _check(code, self._h)
        return F

    def step(self, W, dt=0.0):
        info = SolveInfo()
        used = C.c_double(0.0)
        code = lib().gks_step(self._h, _dev(W, (4, self.nt), "W"), float(dt), C.byref(used), C.byref(info))
        _check(code, self._h)
        return used.value, info.as_dict()

    def limit(self, W, X, threshold: float = 1.0, variables: int = 1, Xout=None):
        """(Xout, n_limited): X limited by the DWBAP limiter (gks_limit);
        variables: LIMIT_CONSERVATIVE (1) or LIMIT_CHARACTERISTIC (2)."""
        import torch
        if Xout is None:
            Xout = torch.empty((4, 5, self.nt), dtype=torch.float64, device=X.device)
        n = C.c_int32(0)
        code = lib().gks_limit(self._h, _dev(W, (4, self.nt), "W"), _dev(X, (4, 5, self.nt), "X"),
                               _dev(Xout, (4, 5, self.nt), "Xout"), float(threshold), int(variables),
                               C.byref(n))
        _check(code, self._h)
        return Xout, int(n.value)

    def limit_noalloc(self, W, X, Xout, threshold: float = 1.0, variables: int = 1):
        """n_limited: Xout = X limited by gks_limit_noalloc (no allocation;
        Xout must be given)."""
        n = C.c_int32(0)
        code = lib().gks_limit_noalloc(self._h, _dev(W, (4, self.nt), "W"), _dev(X, (4, 5, self.nt), "X"),
                                       _dev(Xout, (4, 5, self.nt), "Xout"), float(threshold), int(variables),
                                       C.byref(n))
        _check(code, self._h)
        return int(n.value)

    def apply_precond(self, V, form: int = 0, Z=None):
        """Z = P(V) with the solver's preconditioner (gks_apply_precond)."""
        import torch
        if Z is None:
            Z = torch.empty((4, 5, self.nt), dtype=torch.float64, device=V.device)
        code = lib().gks_apply_precond(self._h, _dev(V, (4, 5, self.nt), "V"), _dev(Z, (4, 5, self.nt), "Z"),
                                       int(form))
        _check(code, self._h)
        return Z

    def profile(self, enable: bool):
        _check(lib().gks_profile_enable(self._h, int(enable)), self._h)

    def profile_get(self) -> dict:
        n = 32
        names = (C.c_char_p * n)()
        launches = (C.c_int64 * n)()
        ms = (C.c_double * n)()
        by = (C.c_double * n)()
        k = lib().gks_profile_get(self._h, n, names, launches, ms, by)
        if k < 0:
            _check(k, self._h)
        return {names[i].decode(): {"launches": int(launches[i]), "ms": float(ms[i]), "bytes": float(by[i])}
                for i in range(k) if names[i]}


class GksBatch:
    """A batch context (gks_batch): one step of several mesh handles at once
    in shared grouped launches, each handle's result bitwise that of its own
    eager step."""

    MAX = 64

    def __init__(self, stream=None):
        self._b = None
        if stream is None:
            import torch
            stream = torch.cuda.current_stream()
        self.stream = stream
        sp = C.c_void_p(int(getattr(stream, "cuda_stream", stream) or 0))
        b = C.c_void_p()
        code = lib().gks_batch_create(sp, C.byref(b))
        if code != GKS_OK:
            raise GksError(code, "gks_batch_create failed")
        self._b = b

    def close(self):
        if self._b is not None:
            lib().gks_batch_destroy(self._b)
            self._b = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def step(self, meshes, states, dt=None):
        """One step of each (GksMesh, W) pair.  Returns a list of
        (status code, dt used, info dict); a handle whose step failed keeps
        its W, as gks_step (status GKS_ENOCONV or GKS_ENONPHYS)."""
        n = len(meshes)
        if n != len(states) or not 1 <= n <= self.MAX:
            raise ValueError("1 to %d (mesh, W) pairs" % self.MAX)
        hs = (C.c_void_p * n)(*[m._h for m in meshes])
        ws = (C.c_void_p * n)(*[_dev(W, (4, m.nt), "W") for m, W in zip(meshes, states)])
        dts = (C.c_double * n)(*([0.0] * n if dt is None else [float(x) for x in dt]))
        used = (C.c_double * n)()
        infos = (SolveInfo * n)()
        st = (C.c_int32 * n)()
        code = lib().gks_batch_step(self._b, n, hs, ws, dts, used, infos, st)
        if code != GKS_OK:
            raise GksError(code, lib().gks_batch_last_error(self._b).decode(errors="replace"))
        return [(int(st[r]), float(used[r]), infos[r].as_dict()) for r in range(n)]
