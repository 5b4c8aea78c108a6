"""Python binding of the nbte C ABI (include/nbte.h): argument marshalling only.

Every function named nbte_* here calls the C function of the same name in the
in-tree libnbte.so; there is no Python or CPU implementation of any step.  If
the library is not built, importing this module raises.  torch is used only
to supply the HIP stream and, optionally, device output arrays.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnbte.so")

# --- constants (values of include/nbte.h) ----------------------------------
OK = 0
ERR_INVALID_ARG, ERR_MESH, ERR_QUADRATURE, ERR_BOUNDARY, ERR_ILL_POSED = -1, -2, -3, -4, -5
ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_NOT_CONVERGED, ERR_DIVERGED, ERR_STATE = -6, -7, -8, -9, -10
CELL = {"tri3": 1, "quad4": 2, "tet4": 3, "hex8": 4}
BC = {"thermalizing": 1, "specular": 2, "diffuse": 3, "partial": 4}
SCHEME = {"sequential": 0, "synthetic": 1, "synthetic_literal": 2}
PRECISION = {"fp64": 0, "mixed": 1}

_d = ct.POINTER(ct.c_double)
_i64 = ct.POINTER(ct.c_int64)
_i32 = ct.POINTER(ct.c_int32)


class Boundary(ct.Structure):
    _fields_ = [("tag", ct.c_int32), ("kind", ct.c_int32), ("T_wall", ct.c_double), ("specularity", ct.c_double)]


class SolveOpts(ct.Structure):
    _fields_ = [("scheme", ct.c_int32), ("precision", ct.c_int32), ("T_ref", ct.c_double), ("tol", ct.c_double),
                ("max_iter", ct.c_int32), ("check_every", ct.c_int32), ("T_init", _d),
                ("outputs_on_device", ct.c_int32), ("time_phases", ct.c_int32), ("refine", ct.c_int32),
                ("spatial_order", ct.c_int32)]


class Result(ct.Structure):
    _fields_ = [("T_lattice", _d), ("T", _d), ("q", _d), ("iterations", ct.c_int32), ("residual", ct.c_double),
                ("energy_defect", ct.c_double)]


class MeshInfo(ct.Structure):
    _fields_ = [("dim", ct.c_int32), ("faces_per_cell", ct.c_int32), ("n_cells", ct.c_int64),
                ("n_bfaces", ct.c_int64), ("total_volume", ct.c_double), ("max_closure_error", ct.c_double)]


class Stats(ct.Structure):
    _fields_ = [("iterations", ct.c_int32), ("ms_total", ct.c_double), ("ms_bc", ct.c_double),
                ("ms_sweep", ct.c_double), ("ms_moments", ct.c_double), ("ms_synthetic", ct.c_double),
                ("ms_update", ct.c_double), ("sweep_launches", ct.c_int32), ("updates_per_sweep", ct.c_int64),
                ("max_levels", ct.c_int32), ("device_bytes", ct.c_int64), ("bands_per_block", ct.c_int32),
                ("bands_per_lane", ct.c_int32), ("block_size", ct.c_int32), ("lds_slots", ct.c_int32),
                ("spilled_values", ct.c_int64), ("refined_at", ct.c_int32)]


class BatchInfo(ct.Structure):
    _fields_ = [("members", ct.c_int32), ("budget_bytes", ct.c_int64), ("bytes_in_use", ct.c_int64),
                ("iterations_launched", ct.c_int64)]


class Tuning(ct.Structure):
    _fields_ = [("bands_per_block", ct.c_int32), ("bands_per_lane", ct.c_int32), ("block_size", ct.c_int32),
                ("lds_bytes", ct.c_int32), ("cg_max_iter", ct.c_int32), ("cg_rtol", ct.c_double),
                ("no_graphs", ct.c_int32), ("accel_depth", ct.c_int32), ("inner_solver", ct.c_int32),
                ("inner_max_iter", ct.c_int32), ("inner_rtol", ct.c_double), ("layout", ct.c_int32)]


# (name, restype, argtypes) of every exported symbol declared in include/nbte.h
SIGNATURES = [
    ("nbte_mesh_create", ct.c_int32, [ct.c_int32, ct.c_int64, _d, ct.c_int32, ct.c_int64, _i64, ct.c_int64, _i64,
                                      _i32, ct.POINTER(ct.c_void_p)]),
    ("nbte_mesh_destroy", None, [ct.c_void_p]),
    ("nbte_mesh_read_gmsh", ct.c_int32, [ct.c_char_p, ct.c_double, ct.POINTER(ct.c_void_p)]),
    ("nbte_mesh_get_regions", ct.c_int32, [ct.c_void_p, _i32]),
    ("nbte_mesh_get_centroids", ct.c_int32, [ct.c_void_p, _d]),
    ("nbte_mesh_get_info", ct.c_int32, [ct.c_void_p, ct.POINTER(MeshInfo)]),
    ("nbte_problem_create", ct.c_int32, [ct.c_void_p, ct.c_void_p, ct.POINTER(ct.c_void_p)]),
    ("nbte_problem_destroy", None, [ct.c_void_p]),
    ("nbte_set_bands", ct.c_int32, [ct.c_void_p, ct.c_int32, _d, _d, _d]),
    ("nbte_set_quadrature", ct.c_int32, [ct.c_void_p, ct.c_int32, _d, _d]),
    ("nbte_set_boundaries", ct.c_int32, [ct.c_void_p, ct.c_int32, ct.POINTER(Boundary)]),
    ("nbte_solve_opts_default", None, [ct.POINTER(SolveOpts)]),
    ("nbte_solve_steady", ct.c_int32, [ct.c_void_p, _d, ct.POINTER(SolveOpts), ct.POINTER(Result)]),
    ("nbte_prepare", ct.c_int32, [ct.c_void_p, _d, ct.POINTER(SolveOpts)]),
    ("nbte_iterate", ct.c_int32, [ct.c_void_p, ct.c_int32, ct.c_int32, _d]),
    ("nbte_read_result", ct.c_int32, [ct.c_void_p, ct.POINTER(Result)]),
    ("nbte_get_distribution", ct.c_int32, [ct.c_void_p, ct.c_int32, ct.c_int32, _d]),
    ("nbte_get_distribution_noalloc", ct.c_int32, [ct.c_void_p, ct.c_int32, ct.c_int32, _d]),
    ("nbte_get_lagged_faces", ct.c_int32, [ct.c_void_p, ct.c_int32, _i32, _i32, ct.c_int32, _i32]),
    ("nbte_get_schedule", ct.c_int32, [ct.c_void_p, ct.c_int32, _i32, _i32, ct.c_int32, _i32]),
    ("nbte_get_stats", ct.c_int32, [ct.c_void_p, ct.POINTER(Stats)]),
    ("nbte_set_tuning", ct.c_int32, [ct.c_void_p, ct.POINTER(Tuning)]),
    ("nbte_get_tuning", ct.c_int32, [ct.c_void_p, ct.POINTER(Tuning)]),
    ("nbte_problem_footprint", ct.c_int32, [ct.c_void_p, ct.c_int32, _i64]),
    ("nbte_problem_setup", ct.c_int32, [ct.c_void_p, ct.c_int32]),
    ("nbte_batch_create", ct.c_int32, [ct.c_void_p, ct.c_int64, ct.POINTER(ct.c_void_p)]),
    ("nbte_batch_destroy", None, [ct.c_void_p]),
    ("nbte_batch_admit", ct.c_int32, [ct.c_void_p, ct.c_void_p, _d, ct.POINTER(SolveOpts)]),
    ("nbte_batch_step", ct.c_int32, [ct.c_void_p, ct.c_int32]),
    ("nbte_batch_poll", ct.c_int32, [ct.c_void_p, ct.POINTER(ct.c_void_p), ct.c_int32, _i32, _i32]),
    ("nbte_batch_remove", ct.c_int32, [ct.c_void_p, ct.c_void_p]),
    ("nbte_batch_get_info", ct.c_int32, [ct.c_void_p, ct.POINTER(BatchInfo)]),
    ("nbte_last_error", ct.c_char_p, []),
    ("nbte_version", ct.c_char_p, []),
]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    # One HIP runtime per process: torch ships its own libamdhip64 (same
    # SONAME).  Loading torch first lets libnbte.so bind to that instance;
    # loading libnbte.so first would pull in a second HIP/HSA runtime, which
    # then finds no device.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ct.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


class NbteError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"nbte status {status}: {message}")
        self.status = status
        self.message = message


def _check(status):
    if status != OK:
        raise NbteError(status, (_lib.nbte_last_error() or b"").decode())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=_d):
    return a.ctypes.data_as(t)


def _stream(stream):
    if stream is not None:
        return ct.c_void_p(int(stream))
    try:
        import torch
        if torch.cuda.is_available():
            return ct.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return ct.c_void_p(0)


class Mesh:
    """Owning wrapper of an nbte_mesh handle."""

    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        # at interpreter exit the module's globals may already be gone: the
        # process's end then releases the handle
        if getattr(self, "handle", None) and _lib is not None:
            _lib.nbte_mesh_destroy(self.handle)
            self.handle = None


class ProblemHandle:
    """Owning wrapper of an nbte_problem handle."""

    def __init__(self, handle, n_cells):
        self.handle = handle
        self.n_cells = n_cells

    def __del__(self):
        # at interpreter exit the module's globals may already be gone: the
        # process's end then releases the handle
        if getattr(self, "handle", None) and _lib is not None:
            _lib.nbte_problem_destroy(self.handle)
            self.handle = None


# --- C ABI, one wrapper per function ----------------------------------------

def nbte_version():
    return _lib.nbte_version().decode()


def nbte_last_error():
    return (_lib.nbte_last_error() or b"").decode()


def nbte_mesh_create(dim, xyz, cell_type, cells, bfaces, bface_tag):
    xyz = _f64(xyz)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    bfaces = np.ascontiguousarray(bfaces, dtype=np.int64)
    tags = np.ascontiguousarray(bface_tag, dtype=np.int32)
    ct_code = CELL[cell_type] if isinstance(cell_type, str) else int(cell_type)
    h = ct.c_void_p()
    _check(_lib.nbte_mesh_create(int(dim), xyz.shape[0], _ptr(xyz), ct_code, cells.shape[0], _ptr(cells, _i64),
                                 bfaces.shape[0], _ptr(bfaces, _i64), _ptr(tags, _i32), ct.byref(h)))
    return Mesh(h)


def nbte_mesh_read_gmsh(path, scale=1.0):
    h = ct.c_void_p()
    _check(_lib.nbte_mesh_read_gmsh(os.fsencode(path), float(scale), ct.byref(h)))
    return Mesh(h)


def nbte_mesh_get_regions(mesh):
    n = nbte_mesh_get_info(mesh)["n_cells"]
    out = np.empty(n, np.int32)
    _check(_lib.nbte_mesh_get_regions(mesh.handle, _ptr(out, _i32)))
    return out


def nbte_mesh_get_centroids(mesh):
    n = nbte_mesh_get_info(mesh)["n_cells"]
    out = np.empty((n, 3))
    _check(_lib.nbte_mesh_get_centroids(mesh.handle, _ptr(out)))
    return out


def nbte_mesh_get_info(mesh):
    info = MeshInfo()
    _check(_lib.nbte_mesh_get_info(mesh.handle, ct.byref(info)))
    return {k: getattr(info, k) for k, _ in MeshInfo._fields_}


def nbte_problem_create(mesh, stream=None):
    h = ct.c_void_p()
    _check(_lib.nbte_problem_create(mesh.handle, _stream(stream), ct.byref(h)))
    return ProblemHandle(h, nbte_mesh_get_info(mesh)["n_cells"])


def nbte_set_bands(p, C, v, tau):
    C, v, tau = _f64(C), _f64(v), _f64(tau)
    _check(_lib.nbte_set_bands(p.handle, len(C), _ptr(C), _ptr(v), _ptr(tau)))


def nbte_set_quadrature(p, s, w):
    s, w = _f64(s).reshape(-1, 3), _f64(w)
    _check(_lib.nbte_set_quadrature(p.handle, len(w), _ptr(s), _ptr(w)))


def nbte_set_boundaries(p, bcs):
    """bcs: iterable of (tag, kind, T_wall, specularity); kind a name or code."""
    arr = (Boundary * len(bcs))()
    for k, (tag, kind, Tw, sp) in enumerate(bcs):
        arr[k] = Boundary(int(tag), BC[kind] if isinstance(kind, str) else int(kind), float(Tw), float(sp))
    _check(_lib.nbte_set_boundaries(p.handle, len(bcs), arr))


def nbte_solve_opts_default():
    o = SolveOpts()
    _lib.nbte_solve_opts_default(ct.byref(o))
    return o


def make_opts(scheme="synthetic", precision="fp64", T_ref=300.0, tol=1e-8, max_iter=10000, check_every=8,
              T_init=None, outputs_on_device=False, time_phases=False, refine=True, order=1):
    o = nbte_solve_opts_default()
    o.scheme = SCHEME[scheme] if isinstance(scheme, str) else int(scheme)
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.T_ref, o.tol, o.max_iter, o.check_every = float(T_ref), float(tol), int(max_iter), int(check_every)
    o.outputs_on_device = int(bool(outputs_on_device))
    o.time_phases = int(bool(time_phases))
    o.refine = int(bool(refine))
    o.spatial_order = int(order)
    o._keep = None
    if T_init is not None:
        t = _f64(T_init)
        o._keep = t
        o.T_init = _ptr(t)
    return o


def _result_buffers(n, on_device):
    if on_device:
        import torch
        bufs = [torch.empty(n, dtype=torch.float64, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda"),
                torch.empty(3 * n, dtype=torch.float64, device="cuda")]
        ptrs = [ct.cast(ct.c_void_p(b.data_ptr()), _d) for b in bufs]
    else:
        bufs = [np.empty(n), np.empty(n), np.empty(3 * n)]
        ptrs = [_ptr(b) for b in bufs]
    r = Result(ptrs[0], ptrs[1], ptrs[2], 0, 0.0, 0.0)
    return r, bufs


def _unpack(r, bufs, on_device):
    q = bufs[2].reshape(-1, 3) if not on_device else bufs[2].view(-1, 3)
    return {"T_lattice": bufs[0], "T": bufs[1], "q": q, "iterations": r.iterations, "residual": r.residual,
            "energy_defect": r.energy_defect}


def nbte_solve_steady(p, Q_cell, opts, allow_not_converged=False):
    Q = None if Q_cell is None else _f64(Q_cell)
    r, bufs = _result_buffers(p.n_cells, bool(opts.outputs_on_device))
    st = _lib.nbte_solve_steady(p.handle, None if Q is None else _ptr(Q), ct.byref(opts), ct.byref(r))
    if st == ERR_NOT_CONVERGED and allow_not_converged:
        out = _unpack(r, bufs, bool(opts.outputs_on_device))
        out["converged"] = False
        return out
    _check(st)
    out = _unpack(r, bufs, bool(opts.outputs_on_device))
    out["converged"] = True
    return out


def nbte_prepare(p, Q_cell, opts):
    Q = None if Q_cell is None else _f64(Q_cell)
    _check(_lib.nbte_prepare(p.handle, None if Q is None else _ptr(Q), ct.byref(opts)))
    p._outputs_on_device = bool(opts.outputs_on_device)


def nbte_iterate(p, n, check=False):
    res = ct.c_double(0.0)
    _check(_lib.nbte_iterate(p.handle, int(n), int(bool(check)), ct.byref(res)))
    return res.value if check else None


def nbte_read_result(p):
    on_dev = getattr(p, "_outputs_on_device", False)
    r, bufs = _result_buffers(p.n_cells, on_dev)
    _check(_lib.nbte_read_result(p.handle, ct.byref(r)))
    return _unpack(r, bufs, on_dev)


def nbte_get_distribution(p, band, direction):
    out = np.empty(p.n_cells)
    _check(_lib.nbte_get_distribution(p.handle, int(band), int(direction), _ptr(out)))
    return out


def nbte_get_distribution_noalloc(p, band, direction):
    out = np.empty(p.n_cells)
    _check(_lib.nbte_get_distribution_noalloc(p.handle, int(band), int(direction), _ptr(out)))
    return out


def nbte_get_schedule(p, direction):
    n = ct.c_int32(0)
    _check(_lib.nbte_get_schedule(p.handle, int(direction), None, None, 0, ct.byref(n)))
    perm = np.empty(p.n_cells, np.int32)
    lvl = np.empty(n.value + 1, np.int32)
    _check(_lib.nbte_get_schedule(p.handle, int(direction), _ptr(perm, _i32), _ptr(lvl, _i32), len(lvl), ct.byref(n)))
    return perm, lvl


def nbte_get_lagged_faces(p, direction):
    n = ct.c_int32(0)
    _check(_lib.nbte_get_lagged_faces(p.handle, int(direction), None, None, 0, ct.byref(n)))
    cells = np.empty(n.value, np.int32)
    faces = np.empty(n.value, np.int32)
    _check(_lib.nbte_get_lagged_faces(p.handle, int(direction), _ptr(cells, _i32), _ptr(faces, _i32), n.value,
                                      ct.byref(n)))
    return cells, faces


def nbte_get_stats(p):
    s = Stats()
    _check(_lib.nbte_get_stats(p.handle, ct.byref(s)))
    return {k: getattr(s, k) for k, _ in Stats._fields_}


def nbte_set_tuning(p, bands_per_block=0, bands_per_lane=0, block_size=0, lds_bytes=0, cg_max_iter=0, cg_rtol=0.0,
                    no_graphs=0, accel_depth=0, inner_solver=0, inner_max_iter=0, inner_rtol=0.0, layout=0):
    t = Tuning(int(bands_per_block), int(bands_per_lane), int(block_size), int(lds_bytes), int(cg_max_iter),
               float(cg_rtol), int(no_graphs), int(accel_depth), int(inner_solver), int(inner_max_iter),
               float(inner_rtol), int(layout))
    _check(_lib.nbte_set_tuning(p.handle, ct.byref(t)))


def nbte_get_tuning(p):
    t = Tuning()
    _check(_lib.nbte_get_tuning(p.handle, ct.byref(t)))
    return {k: getattr(t, k) for k, _ in Tuning._fields_}


def nbte_problem_footprint(p, precision="mixed"):
    b = ct.c_int64(0)
    _check(_lib.nbte_problem_footprint(p.handle, PRECISION[precision] if isinstance(precision, str) else int(precision),
                                       ct.byref(b)))
    return b.value


def nbte_problem_setup(p, precision="mixed"):
    _check(_lib.nbte_problem_setup(p.handle, PRECISION[precision] if isinstance(precision, str) else int(precision)))


class Batch:
    """Owning wrapper of an nbte_batch handle; holds its members' wrappers."""

    def __init__(self, handle):
        self.handle = handle
        self.members = {}

    def __del__(self):
        # at interpreter exit the module's globals may already be gone: the
        # process's end then releases the handle
        if getattr(self, "handle", None) and _lib is not None:
            _lib.nbte_batch_destroy(self.handle)
            self.handle = None


def nbte_batch_create(budget_bytes=0, stream=None):
    h = ct.c_void_p()
    _check(_lib.nbte_batch_create(_stream(stream), int(budget_bytes), ct.byref(h)))
    return Batch(h)


def nbte_batch_admit(b, p, Q_cell, opts):
    Q = None if Q_cell is None else _f64(Q_cell)
    _check(_lib.nbte_batch_admit(b.handle, p.handle, None if Q is None else _ptr(Q), ct.byref(opts)))
    p._outputs_on_device = bool(opts.outputs_on_device)
    b.members[p.handle.value] = p


def nbte_batch_step(b, n):
    _check(_lib.nbte_batch_step(b.handle, int(n)))


def nbte_batch_poll(b):
    """Returns (stopped member wrappers, number still running)."""
    cap = max(len(b.members), 1)
    arr = (ct.c_void_p * cap)()
    nd, nr = ct.c_int32(0), ct.c_int32(0)
    _check(_lib.nbte_batch_poll(b.handle, arr, cap, ct.byref(nd), ct.byref(nr)))
    return [b.members[arr[k]] for k in range(nd.value)], nr.value


def nbte_batch_remove(b, p):
    _check(_lib.nbte_batch_remove(b.handle, p.handle))
    b.members.pop(p.handle.value, None)


def nbte_batch_get_info(b):
    info = BatchInfo()
    _check(_lib.nbte_batch_get_info(b.handle, ct.byref(info)))
    return {k: getattr(info, k) for k, _ in BatchInfo._fields_}


# --- convenience: a whole problem description in one call -------------------

def build_problem(problem, stream=None, mesh=None):
    """problem: any object with the attributes of a steady-solve request
    (dim, xyz, cell_type, cells, bfaces, bface_tag, boundaries, C, v, tau, s, w);
    mesh: an existing mesh handle (e.g. nbte_mesh_read_gmsh) to use instead of
    the problem's arrays.  Returns (mesh, problem handle)."""
    if mesh is None:
        mesh = nbte_mesh_create(problem.dim, problem.xyz, problem.cell_type, problem.cells, problem.bfaces,
                                problem.bface_tag)
    p = nbte_problem_create(mesh, stream)
    nbte_set_bands(p, problem.C, problem.v, problem.tau)
    nbte_set_quadrature(p, problem.s, problem.w)
    nbte_set_boundaries(p, [(b.tag, b.kind, b.T_wall, b.specularity) for b in problem.boundaries])
    return mesh, p


def solve(problem, precision=None, scheme=None, tol=1e-8, max_iter=10000, check_every=8, T_init=None,
          stream=None, allow_not_converged=False, tuning=None, accel=None, order=1):
    """tuning: None (library defaults), "auto" (autotuner cache, defaults if
    the workload was never tuned) or a dict of nbte_set_tuning arguments;
    accel: Anderson depth of the outer iteration (overrides the tuning's)."""
    mesh, p = build_problem(problem, stream)
    precision = precision or problem.precision
    if tuning == "auto":
        from . import tune
        tuning = tune.settings(problem, precision, p)
    if accel is not None:
        tuning = dict(tuning or {}, accel_depth=int(accel))
    if tuning:
        nbte_set_tuning(p, **tuning)
    opts = make_opts(scheme=scheme or problem.scheme, precision=precision,
                     T_ref=problem.T_ref, tol=tol, max_iter=max_iter, check_every=check_every, T_init=T_init,
                     order=order)
    out = nbte_solve_steady(p, problem.Q, opts, allow_not_converged=allow_not_converged)
    out["_handles"] = (mesh, p)
    return out
