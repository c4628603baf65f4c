"""Python binding of libpbm, the MI355X boundary-element Poisson-Boltzmann library.

Argument marshalling only: every step of the computation runs in the HIP
library behind the C ABI declared in ``include/pbm.h``; the functions below
carry the same names.  There is no fallback: importing works anywhere, but
every call raises if ``libpbm.so`` is missing or no GPU is usable.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpbm.so")

PB_OK = 0
PB_NOT_CONVERGED = 1
PB_E_INVALID_ARG = -1
PB_E_MESH = -2
PB_E_CHARGES = -3
PB_E_NOMEM = -4
PB_E_DEVICE = -5
PB_E_STATE = -6

PB_DIRECT_INT = 0
PB_JUFFER = 1
PB_DIRECT_EXT = 2
PB_DIRECT_INT_PERM = 3
PB_DIRECT_EXT_PERM = 4
PB_MULLER_INT = 5
PB_MULLER_EXT = 6
PB_LU = 7
PB_PMCHWT_INT = 8
PB_PMCHWT_EXT = 9
PB_CFIE_INT = 10
PB_CFIE_EXT = 11
PB_PREC_NONE = 0
PB_BLOCK_DIAG = 1
PB_MASS = 2
PB_SCALED_MASS = 3
PB_CALDERON = 4
PB_CALDERON_INT = 5
PB_CALDERON_EXT = 6
PB_SCALED_CALDERON_INT = 7
PB_SCALED_CALDERON_EXT = 8
PB_FP64 = 0
PB_FP32 = 1
PB_MIXED_BF16 = 2
PB_MIXED_FP16 = 3
PB_MATRIX_FREE = 0
PB_ASSEMBLED = 1
PB_AUTO = 2
PB_TREECODE = 3
PB_APPLY_PRECOND = 1
PB_APPLY_FAR_ONLY = 2
PB_APPLY_NEAR_ONLY = 4
PB_MAX_BATCH_REQUESTS = 1024


class PbError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pbm error {code}: {msg}")
        self.code = code


class pb_mesh(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int32), ("n_triangles", ctypes.c_int32),
                ("xyz", ctypes.POINTER(ctypes.c_double)), ("tri", ctypes.POINTER(ctypes.c_int32))]


class pb_charges(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("xyz", ctypes.POINTER(ctypes.c_double)),
                ("q", ctypes.POINTER(ctypes.c_double))]


class pb_options(ctypes.Structure):
    _fields_ = [("eps_in", ctypes.c_double), ("eps_out", ctypes.c_double), ("kappa", ctypes.c_double),
                ("formulation", ctypes.c_int32), ("preconditioner", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("operator_mode", ctypes.c_int32),
                ("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("singular_order", ctypes.c_int32),
                ("source_chunks", ctypes.c_int32), ("inner_max_iter", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("memory_budget", ctypes.c_size_t), ("use_graph", ctypes.c_int32),
                ("calderon_fast", ctypes.c_int32), ("tree_degree", ctypes.c_int32), ("tree_theta", ctypes.c_double),
                ("cfie_alpha", ctypes.c_double), ("cfie_beta", ctypes.c_double), ("regular_order", ctypes.c_int32),
                ("far_symmetric", ctypes.c_int32)]


class pb_result(ctypes.Structure):
    _fields_ = [("phi", ctypes.POINTER(ctypes.c_double)), ("dphi", ctypes.POINTER(ctypes.c_double)),
                ("dG_kcal", ctypes.c_double), ("iterations", ctypes.c_int32),
                ("outer_iterations", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("t_setup", ctypes.c_double), ("t_rhs", ctypes.c_double), ("t_prec", ctypes.c_double),
                ("t_gmres", ctypes.c_double), ("t_dG", ctypes.c_double), ("device_bytes", ctypes.c_size_t)]


class pb_request_times(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_start", ctypes.c_double), ("t_end", ctypes.c_double)]


class pb_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("running", ctypes.c_int32), ("queued", ctypes.c_int32),
                ("peak_running", ctypes.c_int32), ("inflight_bytes", ctypes.c_size_t),
                ("peak_inflight_bytes", ctypes.c_size_t), ("budget", ctypes.c_size_t)]


class pb_mesh_info(ctypes.Structure):
    _fields_ = [("n_vertices", ctypes.c_int32), ("n_triangles", ctypes.c_int32),
                ("n_near_pairs", ctypes.c_int64), ("near_nnz", ctypes.c_int64),
                ("source_chunks", ctypes.c_int32), ("assembled", ctypes.c_int32),
                ("device_bytes", ctypes.c_size_t), ("far_symmetric", ctypes.c_int32)]


EXPORTS = ["pb_default_options", "pb_last_error", "pb_device_count", "pb_solve", "pb_mesh_create",
           "pb_mesh_destroy", "pb_mesh_get_info", "pb_mesh_refresh", "pb_mesh_solve", "pb_solve_multi", "pb_solve_batch", "pb_mesh_apply",
           "pb_mesh_apply_device", "pb_mesh_rhs", "pb_mesh_reaction_potential", "pb_mesh_near_blocks",
           "pb_mesh_preconditioner", "pb_mesh_profile", "pb_mesh_profile_read", "pb_mesh_synchronize",
           "pb_estimate_device_bytes", "pb_server_create", "pb_server_destroy", "pb_submit", "pb_poll", "pb_cancel",
           "pb_wait", "pb_server_get_stats", "pb_mesh_reaction_potential_noalloc"]

_lib = None


def load():
    """Load libpbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2108_10481_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    L.pb_default_options.argtypes = [P(pb_options)]
    L.pb_default_options.restype = None
    L.pb_last_error.restype = ctypes.c_char_p
    L.pb_device_count.restype = ctypes.c_int32
    L.pb_solve.argtypes = [P(pb_mesh), P(pb_charges), P(pb_options), P(pb_result)]
    L.pb_mesh_create.argtypes = [P(pb_mesh), P(pb_options), P(vp)]
    L.pb_mesh_destroy.argtypes = [vp]
    L.pb_mesh_get_info.argtypes = [vp, P(pb_mesh_info)]
    L.pb_mesh_refresh.argtypes = [vp]
    L.pb_mesh_solve.argtypes = [vp, P(pb_charges), P(pb_result)]
    L.pb_solve_multi.argtypes = [vp, ctypes.c_int32, P(pb_charges), P(pb_result)]
    L.pb_solve_batch.argtypes = [ctypes.c_int32, P(vp), P(pb_charges), P(pb_result)]
    L.pb_mesh_apply.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int32]
    L.pb_mesh_apply_device.argtypes = [vp, vp, vp, ctypes.c_int32, vp]
    L.pb_mesh_rhs.argtypes = [vp, P(pb_charges), P(ctypes.c_double)]
    L.pb_mesh_reaction_potential.argtypes = [vp, P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int32,
                                             P(ctypes.c_double), P(ctypes.c_double)]
    L.pb_mesh_reaction_potential_noalloc.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp]
    L.pb_mesh_near_blocks.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int32), P(ctypes.c_int32),
                                      P(ctypes.c_double)]
    L.pb_mesh_preconditioner.argtypes = [vp, P(ctypes.c_double)]
    L.pb_mesh_profile.argtypes = [vp, ctypes.c_int32]
    L.pb_mesh_profile_read.argtypes = [vp, ctypes.c_int32, P(ctypes.c_int64), P(ctypes.c_double),
                                       P(ctypes.c_double)]
    L.pb_mesh_synchronize.argtypes = [vp]
    L.pb_estimate_device_bytes.argtypes = [P(pb_mesh), P(pb_options), P(ctypes.c_size_t)]
    L.pb_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int32, P(vp)]
    L.pb_server_destroy.argtypes = [vp]
    L.pb_submit.argtypes = [vp, P(pb_mesh), P(pb_charges), P(pb_options), P(ctypes.c_uint64)]
    L.pb_poll.argtypes = [vp, ctypes.c_uint64, P(ctypes.c_int32)]
    L.pb_cancel.argtypes = [vp, ctypes.c_uint64]
    L.pb_wait.argtypes = [vp, ctypes.c_uint64, P(pb_result), P(pb_request_times)]
    L.pb_server_get_stats.argtypes = [vp, P(pb_server_stats)]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("pb_default_options", "pb_last_error", "pb_device_count"):
            f.restype = ctypes.c_int32
    _lib = L
    return L


def _check(code: int) -> int:
    if code < 0:
        raise PbError(code, load().pb_last_error().decode())
    return code


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def pb_device_count() -> int:
    return int(load().pb_device_count())


def pb_last_error() -> str:
    return load().pb_last_error().decode()


def pb_default_options(**overrides) -> pb_options:
    o = pb_options()
    load().pb_default_options(ctypes.byref(o))
    for k, v in overrides.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class _Keep:
    """Holds the NumPy arrays behind a ctypes struct for the duration of a call."""

    def __init__(self, *arrays):
        self.arrays = arrays


def _mesh_struct(xyz, tri):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
    m = pb_mesh(xyz.shape[0], tri.shape[0], _dptr(xyz), _iptr(tri))
    return m, _Keep(xyz, tri)


def _charges_struct(xyz, q):
    xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    c = pb_charges(q.shape[0], _dptr(xyz), _dptr(q))
    return c, _Keep(xyz, q)


def _result(nv):
    phi = np.zeros(nv)
    dphi = np.zeros(nv)
    r = pb_result()
    r.phi = _dptr(phi)
    r.dphi = _dptr(dphi)
    return r, phi, dphi


def _result_dict(status, r, phi, dphi):
    return {"status": int(status), "phi": phi, "dphi": dphi, "dG": r.dG_kcal, "iterations": r.iterations,
            "outer_iterations": r.outer_iterations, "rel_residual": r.rel_residual, "t_setup": r.t_setup,
            "t_rhs": r.t_rhs, "t_prec": r.t_prec, "t_gmres": r.t_gmres, "t_dG": r.t_dG,
            "device_bytes": int(r.device_bytes)}


def pb_solve(xyz, tri, qxyz, q, options: pb_options | None = None) -> dict:
    opt = options or pb_default_options()
    m, k1 = _mesh_struct(xyz, tri)
    c, k2 = _charges_struct(qxyz, q)
    r, phi, dphi = _result(m.n_vertices)
    st = _check(load().pb_solve(ctypes.byref(m), ctypes.byref(c), ctypes.byref(opt), ctypes.byref(r)))
    return _result_dict(st, r, phi, dphi)


class MeshHandle:
    """A resident mesh (pb_mesh_create / pb_mesh_destroy)."""

    def __init__(self, xyz, tri, options: pb_options | None = None):
        self.options = options or pb_default_options()
        m, keep = _mesh_struct(xyz, tri)
        h = ctypes.c_void_p()
        _check(load().pb_mesh_create(ctypes.byref(m), ctypes.byref(self.options), ctypes.byref(h)))
        self.h = h
        self.nv = m.n_vertices
        self.nt = m.n_triangles

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _check(load().pb_mesh_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        i = pb_mesh_info()
        _check(load().pb_mesh_get_info(self.h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in pb_mesh_info._fields_}


def pb_mesh_create(xyz, tri, options: pb_options | None = None) -> MeshHandle:
    return MeshHandle(xyz, tri, options)


def pb_mesh_destroy(h: MeshHandle) -> None:
    h.close()


def pb_mesh_get_info(h: MeshHandle) -> dict:
    return h.info()


def pb_mesh_refresh(h: MeshHandle) -> None:
    _check(load().pb_mesh_refresh(h.h))


def pb_mesh_solve(h: MeshHandle, qxyz, q) -> dict:
    c, keep = _charges_struct(qxyz, q)
    r, phi, dphi = _result(h.nv)
    st = _check(load().pb_mesh_solve(h.h, ctypes.byref(c), ctypes.byref(r)))
    return _result_dict(st, r, phi, dphi)


def pb_solve_multi(h: MeshHandle, sets) -> list:
    """sets: list of (qxyz, q).  Returns one result dict per set."""
    n = len(sets)
    cs = (pb_charges * n)()
    keep = []
    for k, (qx, qq) in enumerate(sets):
        c, kp = _charges_struct(qx, qq)
        cs[k] = c
        keep.append(kp)
    rs = (pb_result * n)()
    outs = []
    for k in range(n):
        r, phi, dphi = _result(h.nv)
        rs[k] = r
        outs.append((phi, dphi))
    st = _check(load().pb_solve_multi(h.h, n, cs, rs))
    return [_result_dict(st, rs[k], outs[k][0], outs[k][1]) for k in range(n)]


def pb_solve_batch(handles, sets) -> list:
    """handles: list of matrix-free MeshHandle (distinct, one precision);
    sets: one (qxyz, q) per handle.  The far-field products of all requests run
    fused (one persistent launch per kernel form and GMRES iteration).
    Returns one result dict per request."""
    n = len(handles)
    if len(sets) != n:
        raise ValueError("one charge set per handle")
    hs = (ctypes.c_void_p * max(n, 1))(*[h.h for h in handles])
    cs = (pb_charges * max(n, 1))()
    keep = []
    for k, (qx, qq) in enumerate(sets):
        c, kp = _charges_struct(qx, qq)
        cs[k] = c
        keep.append(kp)
    rs = (pb_result * max(n, 1))()
    outs = []
    for k in range(n):
        r, phi, dphi = _result(handles[k].nv)
        rs[k] = r
        outs.append((phi, dphi))
    st = _check(load().pb_solve_batch(n, hs, cs, rs))
    return [_result_dict(st, rs[k], outs[k][0], outs[k][1]) for k in range(n)]


def pb_mesh_apply(h: MeshHandle, x, flags: int = 0) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.shape != (2 * h.nv,):
        raise ValueError("x must have 2 * n_vertices entries")
    y = np.zeros_like(x)
    _check(load().pb_mesh_apply(h.h, _dptr(x), _dptr(y), int(flags)))
    return y


def pb_mesh_apply_device(h: MeshHandle, x_ptr: int, y_ptr: int, flags: int = 0, stream: int = 0) -> None:
    _check(load().pb_mesh_apply_device(h.h, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr), int(flags),
                                       ctypes.c_void_p(stream)))


def pb_mesh_rhs(h: MeshHandle, qxyz, q) -> np.ndarray:
    c, keep = _charges_struct(qxyz, q)
    b = np.zeros(2 * h.nv)
    _check(load().pb_mesh_rhs(h.h, ctypes.byref(c), _dptr(b)))
    return b


def pb_mesh_reaction_potential(h: MeshHandle, phi, dphi, pts) -> np.ndarray:
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    dphi = np.ascontiguousarray(dphi, dtype=np.float64)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
    out = np.zeros(pts.shape[0])
    _check(load().pb_mesh_reaction_potential(h.h, _dptr(phi), _dptr(dphi), pts.shape[0], _dptr(pts), _dptr(out)))
    return out


def pb_mesh_reaction_potential_noalloc(h: MeshHandle, traces_ptr: int, npts: int, pts_ptr: int, out_ptr: int,
                                       stream: int = 0) -> None:
    """Device-pointer variant that allocates nothing: traces_ptr -> 2 V doubles
    [phi; dphi], pts_ptr -> npts x 3 doubles, out_ptr -> npts doubles."""
    _check(load().pb_mesh_reaction_potential_noalloc(h.h, ctypes.c_void_p(traces_ptr), int(npts),
                                                     ctypes.c_void_p(pts_ptr), ctypes.c_void_p(out_ptr),
                                                     ctypes.c_void_p(stream)))


def pb_mesh_near_blocks(h: MeshHandle, t, s) -> np.ndarray:
    t = np.ascontiguousarray(t, dtype=np.int32)
    s = np.ascontiguousarray(s, dtype=np.int32)
    out = np.zeros((t.shape[0], 4, 3, 3))
    _check(load().pb_mesh_near_blocks(h.h, t.shape[0], _iptr(t), _iptr(s), _dptr(out)))
    return out


def pb_mesh_preconditioner(h: MeshHandle) -> np.ndarray:
    out = np.zeros((h.nv, 2, 2))
    _check(load().pb_mesh_preconditioner(h.h, _dptr(out)))
    return out


def pb_mesh_profile(h: MeshHandle, enable) -> None:
    """enable: bit mask of kinds to time (1: operator product, 2: assembly);
    True means both."""
    mask = 3 if enable is True else (0 if enable is False else int(enable))
    _check(load().pb_mesh_profile(h.h, mask))


def pb_mesh_profile_read(h: MeshHandle, kind: int = 0):
    """Returns (launches, total_ms, total_work) for kind 0 (operator product)
    or 1 (dense assembly)."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    w = ctypes.c_double()
    _check(load().pb_mesh_profile_read(h.h, int(kind), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(w)))
    return int(n.value), float(ms.value), float(w.value)


def pb_mesh_synchronize(h: MeshHandle) -> None:
    _check(load().pb_mesh_synchronize(h.h))


def pb_estimate_device_bytes(xyz, tri, options: pb_options | None = None) -> int:
    m, keep = _mesh_struct(xyz, tri)
    b = ctypes.c_size_t()
    _check(load().pb_estimate_device_bytes(ctypes.byref(m), ctypes.byref(options or pb_default_options()),
                                           ctypes.byref(b)))
    return int(b.value)


class Server:
    """Continuous-batching solve server (pb_server_create / pb_server_destroy)."""

    def __init__(self, hbm_budget: int = 0, max_slots: int = 4):
        h = ctypes.c_void_p()
        _check(load().pb_server_create(int(hbm_budget), int(max_slots), ctypes.byref(h)))
        self.h = h
        self.nv = {}

    def submit(self, xyz, tri, qxyz, q, options: pb_options | None = None) -> int:
        m, k1 = _mesh_struct(xyz, tri)
        c, k2 = _charges_struct(qxyz, q)
        t = ctypes.c_uint64()
        _check(load().pb_submit(self.h, ctypes.byref(m), ctypes.byref(c),
                                ctypes.byref(options or pb_default_options()), ctypes.byref(t)))
        self.nv[t.value] = m.n_vertices
        return int(t.value)

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int32()
        _check(load().pb_poll(self.h, ctypes.c_uint64(ticket), ctypes.byref(d)))
        return bool(d.value)

    def cancel(self, ticket: int) -> None:
        _check(load().pb_cancel(self.h, ctypes.c_uint64(ticket)))

    def wait(self, ticket: int) -> dict:
        r, phi, dphi = _result(self.nv.pop(ticket))
        tm = pb_request_times()
        st = _check(load().pb_wait(self.h, ctypes.c_uint64(ticket), ctypes.byref(r), ctypes.byref(tm)))
        out = _result_dict(st, r, phi, dphi)
        out.update({"t_submit": tm.t_submit, "t_start": tm.t_start, "t_end": tm.t_end})
        return out

    def stats(self) -> dict:
        s = pb_server_stats()
        _check(load().pb_server_get_stats(self.h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in pb_server_stats._fields_}

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            _check(load().pb_server_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pb_server_create(hbm_budget: int = 0, max_slots: int = 4) -> Server:
    return Server(hbm_budget, max_slots)
