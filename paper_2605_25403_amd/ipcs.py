"""ctypes binding of libipcs.so (include/ipcs.h): argument marshalling only.

Function names match the C ABI. Device memory for a run is a torch uint8
tensor on the GPU (the run's workspace) and work is issued on a torch stream;
every step of the solver runs in the library's HIP kernels. There is no
fallback: if the library is missing or fails to load, importing this module
raises.
"""
import ctypes as C
import os

import numpy as np
# torch is imported before the library is loaded: torch bundles its own HIP
# runtime, and the library's libamdhip64.so.7 dependency must bind to that same
# already-loaded runtime (one HIP/HSA runtime per process).
import torch  # noqa: F401

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libipcs.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with "
                      "`python -m paper_2605_25403_amd.build` (or __graft_entry__.build())")
lib = C.CDLL(_LIB_PATH)

# ---------------------------------------------------------------- constants
IPCS_OK, IPCS_E_INVALID, IPCS_E_NOMEM, IPCS_E_DEVICE = 0, -1, -2, -3
IPCS_E_NOT_CONVERGED, IPCS_E_BREAKDOWN, IPCS_E_NONFINITE = -4, -5, -6
IPCS_E_STATE, IPCS_E_CAPACITY = -7, -8
IPCS_SPACE_P1, IPCS_SPACE_P2 = 1, 2
IPCS_PAIR_P2P1, IPCS_PAIR_P3P2 = 0, 1
IPCS_PATTERN_P2P2, IPCS_PATTERN_P1P1, IPCS_PATTERN_P1P2, IPCS_PATTERN_P2P1 = 0, 1, 2, 3
IPCS_FP64, IPCS_MIXED = 0, 1
IPCS_CONV_EXPLICIT, IPCS_CONV_SEMI_IMPLICIT = 0, 1
IPCS_SCHEME_IPCS, IPCS_SCHEME_CHORIN = 0, 1
IPCS_START_ZERO, IPCS_START_PREVIOUS = 0, 1
IPCS_MSTART_EXTRAPOLATED, IPCS_MSTART_STATE = 0, 1
IPCS_SOL_TAYLOR_GREEN_2D, IPCS_SOL_JOHN_2D, IPCS_SOL_BELTRAMI_3D = 1, 2, 3
IPCS_SOL_POLY_STEADY_2D, IPCS_SOL_POLY_STEADY_3D = 4, 5
IPCS_SOL_POLY_CUBIC_2D = 6
IPCS_SOL_STEADY_PAPER_2D = 7
IPCS_SOL_POLY_CUBIC_3D = 8
IPCS_STEADY_RESIDUAL, IPCS_STEADY_INCREMENT = 0, 1
IPCS_PHASE_ASM, IPCS_PHASE_MOMENTUM, IPCS_PHASE_PRESSURE, IPCS_PHASE_CORRECTION = 0, 1, 2, 3
IPCS_FIELD_U, IPCS_FIELD_P, IPCS_FIELD_USTAR, IPCS_FIELD_DP = 0, 1, 2, 3
IPCS_FIELD_RHS_MOM, IPCS_FIELD_RHS_P = 4, 5
IPCS_MAT_M, IPCS_MAT_K, IPCS_MAT_KP, IPCS_MAT_A, IPCS_MAT_E = 0, 1, 2, 3, 4
IPCS_MAT_D0, IPCS_MAT_G0, IPCS_MAT_A_ELIM, IPCS_MAT_M_ELIM = 8, 12, 16, 17
IPCS_KERNEL_PCG_SPMV_P, IPCS_KERNEL_PCG_UPDATE_P, IPCS_KERNEL_ASM_CONV = 0, 1, 2
IPCS_KERNEL_BICG_SPMV, IPCS_KERNEL_PCG_SPMV_M = 3, 4
IPCS_KERNEL_BICG_SPMV_T, IPCS_KERNEL_BICG_UPDATE_S, IPCS_KERNEL_BICG_UPDATE_X = 5, 6, 7
IPCS_KERNEL_PCG_UPDATE_M = 8
IPCS_KERNEL_PCG_FUSED_P = 9
IPCS_KERNEL_ASM_SUM = 10
IPCS_NKERNEL = 11


class IpcsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ipcs error {code}: {msg}")
        self.code = code


class ipcs_counts(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nv", C.c_int64), ("nc", C.c_int64), ("n1", C.c_int64),
                ("n2", C.c_int64), ("nnz", C.c_int64 * 4), ("nb2", C.c_int64)]


class ipcs_params(C.Structure):
    _fields_ = [("nu", C.c_double), ("rho", C.c_double), ("dt", C.c_double), ("t0", C.c_double),
                ("precision", C.c_int32), ("convection", C.c_int32),
                ("tol_mom", C.c_double), ("tol_p", C.c_double), ("tol_corr", C.c_double),
                ("tol_ir", C.c_double), ("maxit", C.c_int32), ("check_every", C.c_int32),
                ("callbacks", C.c_int32), ("poisson_part_rows", C.c_int32),
                ("scheme", C.c_int32), ("poisson_s", C.c_int32),
                ("poisson_start", C.c_int32), ("momentum_start", C.c_int32)]


class ipcs_step_stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("it_mom", C.c_int32 * 3), ("it_p", C.c_int32),
                ("it_corr", C.c_int32 * 3), ("ir_outer", C.c_int32), ("failed_solve", C.c_int32),
                ("checks_p", C.c_int32), ("reserved", C.c_int32),
                ("res_mom", C.c_double * 3), ("res_p", C.c_double), ("res_corr", C.c_double * 3),
                ("t", C.c_double), ("ms_asm", C.c_float), ("ms_mom", C.c_float),
                ("ms_p", C.c_float), ("ms_corr", C.c_float)]

    def as_dict(self):
        return {"status": self.status, "it_mom": list(self.it_mom), "it_p": self.it_p,
                "it_corr": list(self.it_corr), "ir_outer": self.ir_outer,
                "checks_p": self.checks_p,
                "res_mom": list(self.res_mom), "res_p": self.res_p,
                "res_corr": list(self.res_corr), "t": self.t,
                "ms": [self.ms_asm, self.ms_mom, self.ms_p, self.ms_corr]}


class ipcs_steady_params(C.Structure):
    _fields_ = [("nu", C.c_double), ("tol", C.c_double), ("maxit", C.c_int32),
                ("restart", C.c_int32), ("lin_tol", C.c_double), ("lin_maxit", C.c_int32),
                ("inner_maxit", C.c_int32), ("inner_tol", C.c_double)]


class ipcs_steady_stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("newton_steps", C.c_int32), ("lin_it", C.c_int32),
                ("inner_it", C.c_int32), ("rel_change", C.c_double), ("res0", C.c_double),
                ("res", C.c_double), ("ms", C.c_float), ("reserved", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


ipcs_field_fn = C.CFUNCTYPE(None, C.c_void_p, C.c_int32, C.c_int64, C.POINTER(C.c_double),
                            C.c_double, C.POINTER(C.c_double))

_P = C.c_void_p
_SIGS = {
    "ipcs_last_error": (C.c_char_p, []),
    "ipcs_mesh_unit_square": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(_P)]),
    "ipcs_mesh_unit_cube": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(_P)]),
    "ipcs_mesh_unit_cube_pair": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                           C.POINTER(_P)]),
    "ipcs_mesh_from_arrays": (C.c_int, [C.c_int32, C.c_int64, _P, C.c_int64, _P, C.POINTER(_P)]),
    "ipcs_mesh_unit_square_pair": (C.c_int, [C.c_int32, C.c_int32, C.c_int32, C.POINTER(_P)]),
    "ipcs_mesh_from_arrays_pair": (C.c_int, [C.c_int32, C.c_int64, _P, C.c_int64, _P, C.c_int32,
                                             C.POINTER(_P)]),
    "ipcs_mesh_pair": (C.c_int, [_P, C.POINTER(C.c_int32)]),
    "ipcs_mesh_counts": (C.c_int, [_P, C.POINTER(ipcs_counts)]),
    "ipcs_mesh_dof_coords": (C.c_int, [_P, C.c_int32, _P, C.c_int64]),
    "ipcs_mesh_cell_dofs": (C.c_int, [_P, C.c_int32, _P, C.c_int64]),
    "ipcs_mesh_boundary": (C.c_int, [_P, _P, C.c_int64]),
    "ipcs_mesh_pattern": (C.c_int, [_P, C.c_int32, _P, C.c_int64, _P, C.c_int64]),
    "ipcs_mesh_p1_partition": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int64)] + [_P] * 8),
    "ipcs_quadrature_rule": (C.c_int, [C.c_int32, C.POINTER(C.c_int32), _P, _P, C.c_int64]),
    "ipcs_quadrature_rule_pair": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_int32), _P, _P,
                                            C.c_int64]),
    "ipcs_mesh_destroy": (None, [_P]),
    "ipcs_params_default": (None, [C.POINTER(ipcs_params)]),
    "ipcs_run_workspace_bytes": (C.c_int, [_P, C.POINTER(ipcs_params), C.POINTER(C.c_int64)]),
    "ipcs_run_create": (C.c_int, [_P, C.POINTER(ipcs_params), _P, C.c_int64, _P, C.POINTER(_P)]),
    "ipcs_set_viscosity": (C.c_int, [_P, C.c_double]),
    "ipcs_set_time_step": (C.c_int, [_P, C.c_double]),
    "ipcs_set_forcing": (C.c_int, [_P, ipcs_field_fn, _P]),
    "ipcs_set_dirichlet": (C.c_int, [_P, ipcs_field_fn, _P]),
    "ipcs_set_builtin_solution": (C.c_int, [_P, C.c_int32, _P, C.c_int32]),
    "ipcs_set_state": (C.c_int, [_P, _P, _P, C.c_double]),
    "ipcs_advance": (C.c_int, [_P, C.c_int32, _P]),
    "ipcs_step_phase": (C.c_int, [_P, C.c_int32, _P]),
    "ipcs_get_velocity": (C.c_int, [_P, _P, C.c_int64]),
    "ipcs_get_pressure": (C.c_int, [_P, _P, C.c_int64]),
    "ipcs_get_time": (C.c_int, [_P, C.POINTER(C.c_double)]),
    "ipcs_get_field": (C.c_int, [_P, C.c_int32, _P, C.c_int64]),
    "ipcs_export_matrix": (C.c_int, [_P, C.c_int32, _P, C.c_int64, _P, _P, C.c_int64]),
    "ipcs_batch_step": (C.c_int, [_P, C.c_int32, _P, _P]),
    "ipcs_batch_step_noalloc": (C.c_int, [_P, C.c_int32, _P, _P]),
    "ipcs_profile_kernel": (C.c_int, [_P, C.c_int32, C.c_int32, C.POINTER(C.c_double)]),
    "ipcs_kernel_timing": (C.c_int, [_P, C.c_uint32]),
    "ipcs_kernel_times": (C.c_int, [_P, C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int32]),
    "ipcs_poisson_partition": (C.c_int, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int64), C.POINTER(C.c_int32)]),
    "ipcs_run_destroy": (None, [_P]),
    "ipcs_steady_params_default": (None, [C.POINTER(ipcs_steady_params)]),
    "ipcs_steady_workspace_bytes": (C.c_int, [_P, C.POINTER(ipcs_steady_params),
                                              C.POINTER(C.c_int64)]),
    "ipcs_steady_create": (C.c_int, [_P, C.POINTER(ipcs_steady_params), _P, C.c_int64, _P,
                                     C.POINTER(_P)]),
    "ipcs_steady_set_builtin": (C.c_int, [_P, C.c_int32, _P, C.c_int32]),
    "ipcs_steady_set_state": (C.c_int, [_P, _P, _P]),
    "ipcs_steady_step": (C.c_int, [_P, C.POINTER(ipcs_steady_stats)]),
    "ipcs_steady_solve": (C.c_int, [_P, C.POINTER(ipcs_steady_stats)]),
    "ipcs_steady_get_velocity": (C.c_int, [_P, _P, C.c_int64]),
    "ipcs_steady_get_pressure": (C.c_int, [_P, _P, C.c_int64]),
    "ipcs_steady_get_vector": (C.c_int, [_P, C.c_int32, _P, C.c_int64]),
    "ipcs_steady_destroy": (None, [_P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_SIGS)


def _check(rc):
    if rc != IPCS_OK:
        raise IpcsError(rc, lib.ipcs_last_error().decode())
    return rc


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- C-ABI names
def ipcs_last_error():
    return lib.ipcs_last_error().decode()


def ipcs_mesh_unit_square(nx, ny):
    h = C.c_void_p()
    _check(lib.ipcs_mesh_unit_square(nx, ny, C.byref(h)))
    return h


def ipcs_mesh_unit_square_pair(nx, ny, pair):
    h = C.c_void_p()
    _check(lib.ipcs_mesh_unit_square_pair(nx, ny, pair, C.byref(h)))
    return h


def ipcs_mesh_unit_cube(nx, ny, nz):
    h = C.c_void_p()
    _check(lib.ipcs_mesh_unit_cube(nx, ny, nz, C.byref(h)))
    return h


def ipcs_mesh_unit_cube_pair(nx, ny, nz, pair):
    h = C.c_void_p()
    _check(lib.ipcs_mesh_unit_cube_pair(nx, ny, nz, pair, C.byref(h)))
    return h


def ipcs_mesh_from_arrays(x, cells):
    x = np.ascontiguousarray(x, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    h = C.c_void_p()
    _check(lib.ipcs_mesh_from_arrays(x.shape[1], x.shape[0], _ptr(x), cells.shape[0],
                                     _ptr(cells), C.byref(h)))
    return h


def ipcs_mesh_from_arrays_pair(x, cells, pair):
    x = np.ascontiguousarray(x, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int32)
    h = C.c_void_p()
    _check(lib.ipcs_mesh_from_arrays_pair(x.shape[1], x.shape[0], _ptr(x), cells.shape[0],
                                          _ptr(cells), pair, C.byref(h)))
    return h


def ipcs_mesh_pair(m):
    v = C.c_int32()
    _check(lib.ipcs_mesh_pair(m, C.byref(v)))
    return v.value


def ipcs_mesh_counts(m):
    c = ipcs_counts()
    _check(lib.ipcs_mesh_counts(m, C.byref(c)))
    return c


def ipcs_mesh_dof_coords(m, space):
    c = ipcs_mesh_counts(m)
    n = c.n1 if space == IPCS_SPACE_P1 else c.n2
    out = np.empty((n, c.dim), dtype=np.float64)
    _check(lib.ipcs_mesh_dof_coords(m, space, _ptr(out), out.size))
    return out


def ipcs_mesh_cell_dofs(m, space):
    c = ipcs_mesh_counts(m)
    if ipcs_mesh_pair(m) == IPCS_PAIR_P3P2:
        p2, p3 = (6, 10) if c.dim == 2 else (10, 20)
        nl = p2 if space == IPCS_SPACE_P1 else p3
    else:
        nl = c.dim + 1 if space == IPCS_SPACE_P1 else (6 if c.dim == 2 else 10)
    out = np.empty((c.nc, nl), dtype=np.int32)
    _check(lib.ipcs_mesh_cell_dofs(m, space, _ptr(out), out.size))
    return out


def ipcs_mesh_boundary(m):
    c = ipcs_mesh_counts(m)
    out = np.empty(c.n2, dtype=np.uint8)
    _check(lib.ipcs_mesh_boundary(m, _ptr(out), out.size))
    return out


def ipcs_mesh_pattern(m, which):
    c = ipcs_mesh_counts(m)
    nrows = c.n2 if which in (IPCS_PATTERN_P2P2, IPCS_PATTERN_P2P1) else c.n1
    rp = np.empty(nrows + 1, dtype=np.int32)
    col = np.empty(c.nnz[which], dtype=np.int32)
    _check(lib.ipcs_mesh_pattern(m, which, _ptr(rp), rp.size, _ptr(col), col.size))
    return rp, col


def ipcs_mesh_p1_partition(m, rows_max):
    """The P1-P1 row partition for parts of at most rows_max rows: dict of
    numpy arrays perm, part_ptr, halo_ptr, halo, slice_ptr, sptr, lcol, src and
    the largest own + halo count lds_rows."""
    sz = (C.c_int64 * 5)()
    _check(lib.ipcs_mesh_p1_partition(m, rows_max, sz, *([None] * 8)))
    nparts, nhalo, nsl, nent, lds = (int(v) for v in sz)
    c = ipcs_mesh_counts(m)
    out = {"perm": np.empty(c.n1, np.int32), "part_ptr": np.empty(nparts + 1, np.int32),
           "halo_ptr": np.empty(nparts + 1, np.int32), "halo": np.empty(max(nhalo, 1), np.int32),
           "slice_ptr": np.empty(nparts + 1, np.int32), "sptr": np.empty(nsl + 1, np.int32),
           "lcol": np.empty(max(nent, 1), np.uint16), "src": np.empty(max(nent, 1), np.int32)}
    keys = ("perm", "part_ptr", "halo_ptr", "halo", "slice_ptr", "sptr", "lcol", "src")
    _check(lib.ipcs_mesh_p1_partition(m, rows_max, sz, *[_ptr(out[k]) for k in keys]))
    out["halo"] = out["halo"][:nhalo]
    out["lcol"] = out["lcol"][:nent]
    out["src"] = out["src"][:nent]
    out["lds_rows"] = lds
    return out


def ipcs_quadrature_rule(dim):
    nq = C.c_int32()
    _check(lib.ipcs_quadrature_rule(dim, C.byref(nq), None, None, 0))
    lam = np.empty((nq.value, dim + 1))
    w = np.empty(nq.value)
    _check(lib.ipcs_quadrature_rule(dim, C.byref(nq), _ptr(lam), _ptr(w), lam.size))
    return lam, w


def ipcs_quadrature_rule_pair(dim, pair):
    nq = C.c_int32()
    _check(lib.ipcs_quadrature_rule_pair(dim, pair, C.byref(nq), None, None, 0))
    lam = np.empty((nq.value, dim + 1))
    w = np.empty(nq.value)
    _check(lib.ipcs_quadrature_rule_pair(dim, pair, C.byref(nq), _ptr(lam), _ptr(w), lam.size))
    return lam, w


def ipcs_mesh_destroy(m):
    lib.ipcs_mesh_destroy(m)


def ipcs_params_default(**kw):
    p = ipcs_params()
    lib.ipcs_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def ipcs_run_workspace_bytes(m, params):
    b = C.c_int64()
    _check(lib.ipcs_run_workspace_bytes(m, C.byref(params), C.byref(b)))
    return b.value


def ipcs_run_create(m, params, dev_ptr, nbytes, stream_ptr):
    h = C.c_void_p()
    _check(lib.ipcs_run_create(m, C.byref(params), C.c_void_p(dev_ptr), nbytes,
                               C.c_void_p(stream_ptr), C.byref(h)))
    return h


def ipcs_set_viscosity(r, nu):
    _check(lib.ipcs_set_viscosity(r, nu))


def ipcs_set_time_step(r, dt):
    _check(lib.ipcs_set_time_step(r, dt))


def ipcs_set_builtin_solution(r, kind, prm=()):
    a = np.ascontiguousarray(prm, dtype=np.float64)
    _check(lib.ipcs_set_builtin_solution(r, kind, _ptr(a) if a.size else None, a.size))


def ipcs_set_state(r, u, p, t):
    u = np.ascontiguousarray(u, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    _check(lib.ipcs_set_state(r, _ptr(u), _ptr(p), t))


def ipcs_advance(r, nsteps, with_stats=True):
    st = (ipcs_step_stats * max(nsteps, 1))() if with_stats else None
    rc = lib.ipcs_advance(r, nsteps, C.cast(st, C.c_void_p) if st is not None else None)
    if rc != IPCS_OK:
        err = IpcsError(rc, lib.ipcs_last_error().decode())
        err.stats = st
        raise err
    return [s.as_dict() for s in st][:nsteps] if st is not None else None


def ipcs_batch_step(runs, stream):
    """One step of every run handle in runs, with shared launches on stream
    (an int HIP stream handle). Returns (rc, per-run stats dicts); a failed
    solve of some run is reported in rc and its stats, not raised."""
    n = len(runs)
    arr = (_P * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in runs])
    st = (ipcs_step_stats * n)()
    rc = lib.ipcs_batch_step(arr, n, C.c_void_p(stream), C.cast(st, C.c_void_p))
    if rc in (IPCS_E_INVALID, IPCS_E_STATE, IPCS_E_DEVICE, IPCS_E_NOMEM):
        raise IpcsError(rc, lib.ipcs_last_error().decode())
    return rc, [s.as_dict() for s in st]


IPCS_BATCH_SCRATCH_BYTES = 16 << 20
IPCS_BATCH_NOALLOC_MAX_RUNS = 256


def ipcs_batch_step_noalloc(runs, stream):
    """ipcs_batch_step without allocation (the library's fixed descriptor
    array); a batch it cannot hold raises with IPCS_E_CAPACITY before any
    work."""
    n = len(runs)
    arr = (_P * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in runs])
    st = (ipcs_step_stats * n)()
    rc = lib.ipcs_batch_step_noalloc(arr, n, C.c_void_p(stream), C.cast(st, C.c_void_p))
    if rc in (IPCS_E_INVALID, IPCS_E_STATE, IPCS_E_DEVICE, IPCS_E_NOMEM, IPCS_E_CAPACITY):
        raise IpcsError(rc, lib.ipcs_last_error().decode())
    return rc, [s.as_dict() for s in st]


def ipcs_step_phase(r, phase):
    st = ipcs_step_stats()
    _check(lib.ipcs_step_phase(r, phase, C.byref(st)))
    return st.as_dict()


def ipcs_get_time(r):
    t = C.c_double()
    _check(lib.ipcs_get_time(r, C.byref(t)))
    return t.value


def ipcs_get_field(r, which, n):
    out = np.empty(n, dtype=np.float64)
    _check(lib.ipcs_get_field(r, which, _ptr(out), out.size))
    return out


def ipcs_export_matrix(r, which, shape_rows, nnz):
    rp = np.empty(shape_rows + 1, dtype=np.int32)
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    _check(lib.ipcs_export_matrix(r, which, _ptr(rp), rp.size, _ptr(col), _ptr(val), nnz))
    return rp, col, val


def ipcs_profile_kernel(r, kernel, nlaunch):
    us = C.c_double()
    _check(lib.ipcs_profile_kernel(r, kernel, nlaunch, C.byref(us)))
    return us.value


def ipcs_kernel_timing(r, mask):
    _check(lib.ipcs_kernel_timing(r, mask))


def ipcs_kernel_times(r):
    """(ms, launches) per kernel id since the last ipcs_kernel_timing call."""
    ms = (C.c_double * IPCS_NKERNEL)()
    cnt = (C.c_int64 * IPCS_NKERNEL)()
    _check(lib.ipcs_kernel_times(r, ms, cnt, IPCS_NKERNEL))
    return list(ms), list(cnt)


def ipcs_poisson_partition(r):
    """dict(rows_max, nparts, halo_rows, lds_rows) of the run's Poisson CG form
    (rows_max 0: two kernels per iteration)."""
    a, b, d = C.c_int32(), C.c_int32(), C.c_int32()
    h = C.c_int64()
    _check(lib.ipcs_poisson_partition(r, C.byref(a), C.byref(b), C.byref(h), C.byref(d)))
    return {"rows_max": a.value, "nparts": b.value, "halo_rows": h.value, "lds_rows": d.value}


def ipcs_run_destroy(r):
    lib.ipcs_run_destroy(r)


def ipcs_steady_params_default(**kw):
    p = ipcs_steady_params()
    lib.ipcs_steady_params_default(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


# ---------------------------------------------------------------- convenience
class Mesh:
    """Owns an ipcs_mesh handle."""

    def __init__(self, handle):
        self.h = handle
        self.counts = ipcs_mesh_counts(handle)

    @classmethod
    def unit_square(cls, nx, ny=None, pair=IPCS_PAIR_P2P1):
        if pair == IPCS_PAIR_P2P1:
            return cls(ipcs_mesh_unit_square(nx, ny or nx))
        return cls(ipcs_mesh_unit_square_pair(nx, ny or nx, pair))

    @classmethod
    def unit_cube(cls, nx, ny=None, nz=None, pair=IPCS_PAIR_P2P1):
        if pair == IPCS_PAIR_P2P1:
            return cls(ipcs_mesh_unit_cube(nx, ny or nx, nz or nx))
        return cls(ipcs_mesh_unit_cube_pair(nx, ny or nx, nz or nx, pair))

    @classmethod
    def from_arrays(cls, x, cells, pair=IPCS_PAIR_P2P1):
        if pair == IPCS_PAIR_P2P1:
            return cls(ipcs_mesh_from_arrays(x, cells))
        return cls(ipcs_mesh_from_arrays_pair(x, cells, pair))

    @property
    def dim(self):
        return self.counts.dim

    @property
    def pair(self):
        return ipcs_mesh_pair(self.h)

    def __del__(self, _destroy=lib.ipcs_mesh_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


class Run:
    """A run with its workspace held as a torch uint8 tensor on the GPU."""

    def __init__(self, mesh, params=None, stream=None, device="cuda", **kw):
        import torch
        self.mesh = mesh
        self.params = params if params is not None else ipcs_params_default(**kw)
        self.ws_bytes = ipcs_run_workspace_bytes(mesh.h, self.params)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.h = ipcs_run_create(mesh.h, self.params, self.ws.data_ptr(), self.ws_bytes,
                                 self.stream.cuda_stream)
        self.dim, self.n1, self.n2 = mesh.counts.dim, mesh.counts.n1, mesh.counts.n2
        self._keep = []

    def set_builtin(self, kind, prm=()):
        ipcs_set_builtin_solution(self.h, kind, prm)

    def set_state(self, u, p, t):
        ipcs_set_state(self.h, u, p, t)

    def set_dirichlet(self, fn):
        cb = self._wrap(fn)
        _check(lib.ipcs_set_dirichlet(self.h, cb, None))

    def set_forcing(self, fn):
        cb = self._wrap(fn) if fn is not None else ipcs_field_fn()
        _check(lib.ipcs_set_forcing(self.h, cb, None))

    def _wrap(self, fn):
        def c_fn(ctx, dim, npts, x, t, out):
            X = np.ctypeslib.as_array(x, shape=(npts, dim))
            O = np.ctypeslib.as_array(out, shape=(npts, dim))
            O[:] = fn(X, t)
        cb = ipcs_field_fn(c_fn)
        self._keep.append(cb)
        return cb

    def advance(self, n=1):
        return ipcs_advance(self.h, n)

    def phase(self, ph):
        return ipcs_step_phase(self.h, ph)

    def velocity(self):
        return ipcs_get_field(self.h, IPCS_FIELD_U, self.dim * self.n2).reshape(self.dim, self.n2)

    def pressure(self):
        return ipcs_get_field(self.h, IPCS_FIELD_P, self.n1)

    def field(self, which):
        n = self.dim * self.n2 if which in (IPCS_FIELD_U, IPCS_FIELD_USTAR, IPCS_FIELD_RHS_MOM) \
            else self.n1
        v = ipcs_get_field(self.h, which, n)
        return v.reshape(self.dim, self.n2) if n == self.dim * self.n2 else v

    def time(self):
        return ipcs_get_time(self.h)

    def kernel_timing(self, mask):
        ipcs_kernel_timing(self.h, mask)

    def kernel_times(self):
        return ipcs_kernel_times(self.h)

    def poisson_partition(self):
        return ipcs_poisson_partition(self.h)

    def matrix(self, which):
        """(rowptr, col, val) of a device matrix, as a scipy CSR matrix."""
        import scipy.sparse as sp
        c = self.mesh.counts
        if which in (IPCS_MAT_M, IPCS_MAT_K, IPCS_MAT_E, IPCS_MAT_A_ELIM, IPCS_MAT_M_ELIM):
            rows, cols, nnz = c.n2, c.n2, c.nnz[IPCS_PATTERN_P2P2]
        elif which == IPCS_MAT_KP:
            rows, cols, nnz = c.n1, c.n1, c.nnz[IPCS_PATTERN_P1P1]
        elif IPCS_MAT_D0 <= which < IPCS_MAT_D0 + 3:
            rows, cols, nnz = c.n1, c.n2, c.nnz[IPCS_PATTERN_P1P2]
        else:
            rows, cols, nnz = c.n2, c.n1, c.nnz[IPCS_PATTERN_P2P1]
        rp, col, val = ipcs_export_matrix(self.h, which, rows, nnz)
        return sp.csr_matrix((val, col, rp), shape=(rows, cols))

    def __del__(self, _destroy=lib.ipcs_run_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None


class Steady:
    """Steady Navier-Stokes by Newton's method (ipcs_steady_*), its workspace
    held as a torch uint8 tensor on the GPU."""

    def __init__(self, mesh, params=None, stream=None, device="cuda", **kw):
        import torch
        self.mesh = mesh
        self.params = params if params is not None else ipcs_steady_params_default(**kw)
        b = C.c_int64()
        _check(lib.ipcs_steady_workspace_bytes(mesh.h, C.byref(self.params), C.byref(b)))
        self.ws_bytes = b.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = _P()
        _check(lib.ipcs_steady_create(mesh.h, C.byref(self.params), self.ws.data_ptr(),
                                      self.ws_bytes, self.stream.cuda_stream, C.byref(h)))
        self.h = h
        self.dim, self.n1, self.n2 = mesh.counts.dim, mesh.counts.n1, mesh.counts.n2

    def set_builtin(self, kind, prm=()):
        a = np.ascontiguousarray(prm, dtype=np.float64)
        _check(lib.ipcs_steady_set_builtin(self.h, kind, _ptr(a) if a.size else None, a.size))

    def set_state(self, U, P):
        u = np.ascontiguousarray(U, dtype=np.float64).ravel()
        p = np.ascontiguousarray(P, dtype=np.float64)
        _check(lib.ipcs_steady_set_state(self.h, _ptr(u), _ptr(p)))

    def step(self):
        st = ipcs_steady_stats()
        _check(lib.ipcs_steady_step(self.h, C.byref(st)))
        return st.as_dict()

    def solve(self):
        """Newton steps to the tolerance; returns the stats (raises on failure)."""
        st = ipcs_steady_stats()
        rc = lib.ipcs_steady_solve(self.h, C.byref(st))
        if rc != IPCS_OK:
            err = IpcsError(rc, lib.ipcs_last_error().decode())
            err.stats = st.as_dict()
            raise err
        return st.as_dict()

    def velocity(self):
        u = np.empty(self.dim * self.n2)
        _check(lib.ipcs_steady_get_velocity(self.h, _ptr(u), u.size))
        return u.reshape(self.dim, self.n2)

    def pressure(self):
        p = np.empty(self.n1)
        _check(lib.ipcs_steady_get_pressure(self.h, _ptr(p), p.size))
        return p

    def vector(self, which):
        """The last step's residual or increment as (U-part (dim, N2), P-part)."""
        v = np.empty(self.dim * self.n2 + self.n1)
        _check(lib.ipcs_steady_get_vector(self.h, which, _ptr(v), v.size))
        return v[:self.dim * self.n2].reshape(self.dim, self.n2), v[self.dim * self.n2:]

    def __del__(self, _destroy=lib.ipcs_steady_destroy):
        if getattr(self, "h", None):
            _destroy(self.h)
            self.h = None
