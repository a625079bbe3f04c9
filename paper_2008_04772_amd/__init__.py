"""Python binding of libpmchwt.so, the MI355X (gfx950) PMCHWT library.

Argument marshalling only: numpy arrays are passed as plain host pointers to
the C ABI declared in include/pmchwt.h, whose entry points carry the same
names.  Every computation runs in the library's HIP kernels.  Importing this
module fails loudly when the shared library has not been built; there is no
fallback path.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmchwt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libpmchwt.so is not built; run `python paper_2008_04772_amd/build.py` "
        "(or __graft_entry__.build()) first")

_lib = ctypes.CDLL(LIB_PATH)

OK = 0
ERR_INVALID_ARG, ERR_INVALID_MESH, ERR_OUT_OF_MEMORY, ERR_DEVICE = -1, -2, -3, -4
ERR_NOT_CONVERGED, ERR_OVER_BUDGET, ERR_CANCELLED, ERR_STATE = -5, -6, -7, -8
PENDING, RUNNING = 1, 2

PRECOND = {"I": 0, "A": 1, "D": 2, "D_INT": 3, "D_EXT": 4, "S_INT": 5, "S_EXT": 6}
FP64, MIXED = 0, 1
OP_S, OP_C = 0, 1
EXT, INT = 0, 1
RWG, BC = 0, 1


class pmchwt_complex(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class pmchwt_assembly_opts(ctypes.Structure):
    _fields_ = [("q_near", ctypes.c_int32), ("q_medium", ctypes.c_int32), ("q_far", ctypes.c_int32),
                ("n_singular", ctypes.c_int32), ("chi", ctypes.c_double), ("precision", ctypes.c_int32),
                ("mass_method", ctypes.c_int32), ("operator_form", ctypes.c_int32), ("mass_hops", ctypes.c_int32)]


class pmchwt_solver_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("ir_max", ctypes.c_int32)]


class pmchwt_solve_stats(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("matvecs", ctypes.c_int64),
                ("rel_residual", ctypes.c_double), ("ir_steps", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("ms_solve", ctypes.c_double)]


class pmchwt_profile(ctypes.Structure):
    _fields_ = [("ms_assemble_A", ctypes.c_double), ("ms_assemble_regular", ctypes.c_double),
                ("ms_regular_combine", ctypes.c_double),
                ("ms_assemble_singular", ctypes.c_double), ("ms_assemble_P", ctypes.c_double),
                ("ms_mass", ctypes.c_double), ("regular_pairs", ctypes.c_int64),
                ("regular_point_pairs", ctypes.c_int64), ("singular_pairs", ctypes.c_int64),
                ("singular_point_pairs", ctypes.c_int64), ("bary_pairs", ctypes.c_int64),
                ("nnz_P", ctypes.c_int64), ("regular_launches", ctypes.c_int32),
                ("n_wavenumbers", ctypes.c_int32), ("recompute", ctypes.c_double),
                ("wall_setup", ctypes.c_double), ("wall_A", ctypes.c_double), ("wall_P", ctypes.c_double),
                ("wall_mass", ctypes.c_double), ("ms_matvec_total", ctypes.c_double),
                ("matvec_launches", ctypes.c_int64), ("matvec_bytes", ctypes.c_int64),
                ("ms_mfma_total", ctypes.c_double), ("mfma_launches", ctypes.c_int64),
                ("mfma_flops", ctypes.c_int64), ("mass_iterations", ctypes.c_int32),
                ("mass_residual", ctypes.c_double), ("lookahead_discarded", ctypes.c_int64),
                ("ms_matvec_reduce", ctypes.c_double), ("matvec_timed", ctypes.c_int64),
                ("ms_free_apply", ctypes.c_double), ("free_launches", ctypes.c_int64),
                ("wall_tables_A", ctypes.c_double), ("wall_tables_P", ctypes.c_double),
                ("wall_dual", ctypes.c_double), ("ms_fp64_copy", ctypes.c_double)]


class pmchwt_server_opts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_live", ctypes.c_int32)]


class pmchwt_request(ctypes.Structure):
    _fields_ = [("n_scatterers", ctypes.c_int32),
                ("verts", ctypes.POINTER(ctypes.POINTER(ctypes.c_double))),
                ("nv", ctypes.POINTER(ctypes.c_int32)),
                ("tris", ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))),
                ("nt", ctypes.POINTER(ctypes.c_int32)),
                ("eps_r", ctypes.POINTER(pmchwt_complex)),
                ("k_ext", ctypes.c_double), ("nrhs", ctypes.c_int32),
                ("dirs", ctypes.POINTER(ctypes.c_double)), ("pols", ctypes.POINTER(pmchwt_complex)),
                ("opts_A", pmchwt_assembly_opts), ("opts_P", pmchwt_assembly_opts),
                ("precond", ctypes.c_int32), ("solver", pmchwt_solver_opts)]


class pmchwt_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("nrhs", ctypes.c_int32), ("n_unknowns", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("ms_queued", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("stats", pmchwt_solve_stats)]


class pmchwt_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "failed", "live", "pending", "rounds",
                                              "max_live_seen", "grouped_launches", "grouped_jobs",
                                              "bytes_in_use")]


_P = ctypes.c_void_p
_pd = ctypes.POINTER(ctypes.c_double)
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pc = ctypes.POINTER(pmchwt_complex)

_SIGS = {
    "pmchwt_version": ([], ctypes.c_char_p),
    "pmchwt_create": ([ctypes.POINTER(_P), ctypes.c_int, _P], ctypes.c_int),
    "pmchwt_add_scatterer": ([_P, _pd, ctypes.c_int32, _pi32, ctypes.c_int32, pmchwt_complex, _pi32], ctypes.c_int),
    "pmchwt_set_wavenumber": ([_P, ctypes.c_double], ctypes.c_int),
    "pmchwt_sizes": ([_P, _pi32, _pi64], ctypes.c_int),
    "pmchwt_num_edges": ([_P, ctypes.c_int32, _pi32], ctypes.c_int),
    "pmchwt_assemble": ([_P, ctypes.POINTER(pmchwt_assembly_opts), ctypes.POINTER(pmchwt_assembly_opts),
                         ctypes.c_int], ctypes.c_int),
    "pmchwt_get_block": ([_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int32, ctypes.c_int32, _pc,
                          ctypes.c_int64], ctypes.c_int),
    "pmchwt_get_entries": ([_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_int64, _pi32, _pi32, _pc], ctypes.c_int),
    "pmchwt_get_mass": ([_P, ctypes.c_int32, _pd], ctypes.c_int),
    "pmchwt_rhs": ([_P, _pd, _pc, ctypes.c_int32, _pc], ctypes.c_int),
    "pmchwt_apply": ([_P, ctypes.c_int32, _pc, ctypes.c_int32, _pc], ctypes.c_int),
    "pmchwt_solve": ([_P, _pd, _pc, ctypes.c_int32, ctypes.POINTER(pmchwt_solver_opts), _pc,
                      ctypes.POINTER(pmchwt_solve_stats)], ctypes.c_int),
    "pmchwt_far_field": ([_P, _pc, ctypes.c_int32, _pd, ctypes.c_int32, _pc], ctypes.c_int),
    "pmchwt_far_field_noalloc": ([_P, _pc, ctypes.c_int32, _pd, ctypes.c_int32, _pc], ctypes.c_int),
    "pmchwt_apply_device": ([_P, ctypes.c_int32, _P, ctypes.c_int32, _P, _P], ctypes.c_int),
    "pmchwt_solve_device": ([_P, _pd, _pc, ctypes.c_int32, ctypes.POINTER(pmchwt_solver_opts), _P,
                             ctypes.POINTER(pmchwt_solve_stats), _P], ctypes.c_int),
    "pmchwt_far_field_device": ([_P, _P, ctypes.c_int32, _P, ctypes.c_int32, _P, _P], ctypes.c_int),
    "pmchwt_near_field": ([_P, _pc, ctypes.c_int32, _pd, _pc, _pd, ctypes.c_int32, _pc, _pi32], ctypes.c_int),
    "pmchwt_cross_sections": ([_P, _pc, ctypes.c_int32, _pd, _pc, _pd, _pd], ctypes.c_int),
    "pmchwt_bc_fields": ([_pd, ctypes.c_int32, _pi32, ctypes.c_int32, _pi64, _pi32, _pd], ctypes.c_int),
    "pmchwt_get_profile": ([_P, ctypes.POINTER(pmchwt_profile)], ctypes.c_int),
    "pmchwt_last_error": ([_P], ctypes.c_char_p),
    "pmchwt_destroy": ([_P], None),
    "pmchwt_server_create": ([ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(pmchwt_server_opts)], ctypes.c_int),
    "pmchwt_server_submit": ([_P, ctypes.POINTER(pmchwt_request), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
    "pmchwt_server_poll": ([_P, ctypes.c_uint64, ctypes.POINTER(pmchwt_result)], ctypes.c_int),
    "pmchwt_server_wait": ([_P, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(pmchwt_result)], ctypes.c_int),
    "pmchwt_server_fetch": ([_P, ctypes.c_uint64, _pc, _pd, _pd], ctypes.c_int),
    "pmchwt_server_cancel": ([_P, ctypes.c_uint64], ctypes.c_int),
    "pmchwt_server_get_stats": ([_P, ctypes.POINTER(pmchwt_server_stats)], ctypes.c_int),
    "pmchwt_server_destroy": ([_P], None),
}
for _name, (_args, _res) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_SIGS)


class PmchwtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pmchwt error {code}: {msg}")
        self.code = code


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _ptr(a, t):
    return a.ctypes.data_as(t)


def _check(ctx, rc, allow=()):
    if rc != OK and rc not in allow:
        msg = _lib.pmchwt_last_error(ctx) if ctx else b""
        raise PmchwtError(rc, (msg or b"").decode())
    return rc


# ---------------------------------------------------------------------------
# Entry points, same names as the C ABI
# ---------------------------------------------------------------------------

def pmchwt_version():
    return _lib.pmchwt_version().decode()


def pmchwt_create(device=0, stream=None):
    h = _P()
    rc = _lib.pmchwt_create(ctypes.byref(h), int(device), _P(stream) if stream else None)
    if rc != OK:
        raise PmchwtError(rc, "pmchwt_create failed")
    return h


def pmchwt_destroy(ctx):
    _lib.pmchwt_destroy(ctx)


def pmchwt_add_scatterer(ctx, verts, tris, eps_r):
    v = _f64(verts)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    sid = ctypes.c_int32(-1)
    eps = complex(eps_r)
    _check(ctx, _lib.pmchwt_add_scatterer(ctx, _ptr(v, _pd), len(v), _ptr(t, _pi32), len(t),
                                          pmchwt_complex(eps.real, eps.imag), ctypes.byref(sid)))
    return sid.value


def pmchwt_set_wavenumber(ctx, k_ext):
    _check(ctx, _lib.pmchwt_set_wavenumber(ctx, float(k_ext)))


def pmchwt_sizes(ctx):
    ns, nu = ctypes.c_int32(), ctypes.c_int64()
    _check(ctx, _lib.pmchwt_sizes(ctx, ctypes.byref(ns), ctypes.byref(nu)))
    return ns.value, nu.value


def pmchwt_num_edges(ctx, m):
    E = ctypes.c_int32()
    _check(ctx, _lib.pmchwt_num_edges(ctx, int(m), ctypes.byref(E)))
    return E.value


def assembly_opts(q=(4, 3, 2), n_singular=4, chi=-1.0, precision=FP64, mass_method=0, operator_form=0,
                  mass_hops=0):
    return pmchwt_assembly_opts(int(q[0]), int(q[1]), int(q[2]), int(n_singular),
                                float(chi) if chi is not None and np.isfinite(chi) else -1.0, int(precision),
                                int(mass_method), int(operator_form), int(mass_hops))


def pmchwt_assemble(ctx, optsA, optsP, precond="S_INT"):
    kind = PRECOND[precond] if isinstance(precond, str) else int(precond)
    _check(ctx, _lib.pmchwt_assemble(ctx, ctypes.byref(optsA), ctypes.byref(optsP), kind))


def pmchwt_get_block(ctx, op, medium, space, m, l):
    Em, El = pmchwt_num_edges(ctx, m), pmchwt_num_edges(ctx, l)
    out = np.zeros((Em, El), dtype=np.complex128)
    _check(ctx, _lib.pmchwt_get_block(ctx, op, medium, space, m, l, _ptr(out, _pc), El))
    return out


def pmchwt_get_entries(ctx, op, medium, space, m, l, rows, cols):
    r = np.ascontiguousarray(rows, dtype=np.int32)
    c = np.ascontiguousarray(cols, dtype=np.int32)
    out = np.zeros(len(r), dtype=np.complex128)
    _check(ctx, _lib.pmchwt_get_entries(ctx, op, medium, space, m, l, len(r), _ptr(r, _pi32), _ptr(c, _pi32),
                                        _ptr(out, _pc)))
    return out


def pmchwt_get_mass(ctx, m):
    E = pmchwt_num_edges(ctx, m)
    out = np.zeros((E, E))
    _check(ctx, _lib.pmchwt_get_mass(ctx, m, _ptr(out, _pd)))
    return out


def _waves(dirs, pols):
    d = _f64(dirs).reshape(-1, 3)
    p = _c128(pols).reshape(-1, 3)
    if len(d) != len(p):
        raise ValueError("dirs and pols differ in length")
    return d, p


def pmchwt_rhs(ctx, dirs, pols):
    d, p = _waves(dirs, pols)
    _, N = pmchwt_sizes(ctx)
    out = np.zeros((len(d), N), dtype=np.complex128)
    _check(ctx, _lib.pmchwt_rhs(ctx, _ptr(d, _pd), _ptr(p, _pc), len(d), _ptr(out, _pc)))
    return out


def pmchwt_apply(ctx, which, x):
    x = _c128(np.atleast_2d(x))
    y = np.zeros_like(x)
    _check(ctx, _lib.pmchwt_apply(ctx, int(which), _ptr(x, _pc), x.shape[0], _ptr(y, _pc)))
    return y


# Device-pointer forms: vectors are device addresses (ints) of memory from
# the library's own HIP runtime (this process's libamdhip64), of the plain
# forms' sizes and layouts; `stream` a hipStream_t as an int, or None.
def pmchwt_apply_device(ctx, which, x_dev, nrhs, y_dev, stream=None):
    _check(ctx, _lib.pmchwt_apply_device(ctx, int(which), _P(int(x_dev)), int(nrhs), _P(int(y_dev)),
                                         _P(int(stream) if stream else None)))


def pmchwt_solve_device(ctx, dirs, pols, opts, currents_dev, stream=None, allow_not_converged=False):
    d, p = _waves(dirs, pols)
    st = pmchwt_solve_stats()
    allow = (ERR_NOT_CONVERGED,) if allow_not_converged else ()
    _check(ctx, _lib.pmchwt_solve_device(ctx, _ptr(d, _pd), _ptr(p, _pc), len(d), ctypes.byref(opts),
                                         _P(int(currents_dev)), ctypes.byref(st),
                                         _P(int(stream) if stream else None)), allow)
    return st


def pmchwt_far_field_device(ctx, currents_dev, nrhs, obs_dev, nobs, F_dev, stream=None):
    _check(ctx, _lib.pmchwt_far_field_device(ctx, _P(int(currents_dev)), int(nrhs), _P(int(obs_dev)), int(nobs),
                                             _P(int(F_dev)), _P(int(stream) if stream else None)))


def solver_opts(tol=1e-6, restart=200, max_iter=2000, ir_max=0):
    return pmchwt_solver_opts(float(tol), int(restart), int(max_iter), int(ir_max))


def pmchwt_solve(ctx, dirs, pols, opts, allow_not_converged=False):
    d, p = _waves(dirs, pols)
    _, N = pmchwt_sizes(ctx)
    out = np.zeros((len(d), N), dtype=np.complex128)
    st = pmchwt_solve_stats()
    allow = (ERR_NOT_CONVERGED,) if allow_not_converged else ()
    _check(ctx, _lib.pmchwt_solve(ctx, _ptr(d, _pd), _ptr(p, _pc), len(d), ctypes.byref(opts), _ptr(out, _pc),
                                  ctypes.byref(st)), allow)
    return out, st


def pmchwt_far_field(ctx, currents, obs):
    x = _c128(np.atleast_2d(currents))
    o = _f64(obs).reshape(-1, 3)
    F = np.zeros((x.shape[0], len(o), 3), dtype=np.complex128)
    _check(ctx, _lib.pmchwt_far_field(ctx, _ptr(x, _pc), x.shape[0], _ptr(o, _pd), len(o), _ptr(F, _pc)))
    return F


def pmchwt_far_field_noalloc(ctx, currents, obs):
    x = _c128(np.atleast_2d(currents))
    o = _f64(obs).reshape(-1, 3)
    F = np.zeros((x.shape[0], len(o), 3), dtype=np.complex128)
    _check(ctx, _lib.pmchwt_far_field_noalloc(ctx, _ptr(x, _pc), x.shape[0], _ptr(o, _pd), len(o), _ptr(F, _pc)))
    return F


def pmchwt_near_field(ctx, currents, dirs, pols, points):
    x = _c128(np.atleast_2d(currents))
    d, p = _waves(dirs, pols)
    pts = _f64(points).reshape(-1, 3)
    E = np.zeros((x.shape[0], len(pts), 3), dtype=np.complex128)
    reg = np.zeros(len(pts), dtype=np.int32)
    _check(ctx, _lib.pmchwt_near_field(ctx, _ptr(x, _pc), x.shape[0], _ptr(d, _pd), _ptr(p, _pc), _ptr(pts, _pd),
                                       len(pts), _ptr(E, _pc), _ptr(reg, _pi32)))
    return E, reg


def pmchwt_cross_sections(ctx, currents, dirs, pols):
    x = _c128(np.atleast_2d(currents))
    d, p = _waves(dirs, pols)
    se = np.zeros(x.shape[0])
    ss = np.zeros(x.shape[0])
    _check(ctx, _lib.pmchwt_cross_sections(ctx, _ptr(x, _pc), x.shape[0], _ptr(d, _pd), _ptr(p, _pc),
                                           _ptr(se, _pd), _ptr(ss, _pd)))
    return se, ss


def pmchwt_bc_fields(verts, tris):
    """Host-only: (edge ids, child ids, alpha, w) of every BC restriction."""
    v = _f64(verts)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    n = ctypes.c_int64(0)
    rc = _lib.pmchwt_bc_fields(_ptr(v, _pd), len(v), _ptr(t, _pi32), len(t), ctypes.byref(n), None, None)
    if rc != OK:
        raise PmchwtError(rc, "pmchwt_bc_fields failed")
    ids = np.zeros((n.value, 2), dtype=np.int32)
    vals = np.zeros((n.value, 4))
    rc = _lib.pmchwt_bc_fields(_ptr(v, _pd), len(v), _ptr(t, _pi32), len(t), ctypes.byref(n), _ptr(ids, _pi32),
                               _ptr(vals, _pd))
    if rc != OK:
        raise PmchwtError(rc, "pmchwt_bc_fields failed")
    return ids[:, 0], ids[:, 1], vals[:, 0], vals[:, 1:]


def pmchwt_get_profile(ctx):
    p = pmchwt_profile()
    _check(ctx, _lib.pmchwt_get_profile(ctx, ctypes.byref(p)))
    return {f: getattr(p, f) for f, _ in pmchwt_profile._fields_}


class Context:
    """Owns one pmchwt context; methods forward to the entry points above."""

    def __init__(self, device=0, stream=None):
        self.h = pmchwt_create(device, stream)

    def close(self):
        if self.h:
            pmchwt_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def add_scatterer(self, verts, tris, eps_r):
        return pmchwt_add_scatterer(self.h, verts, tris, eps_r)

    def set_wavenumber(self, k):
        pmchwt_set_wavenumber(self.h, k)

    def sizes(self):
        return pmchwt_sizes(self.h)

    def num_edges(self, m):
        return pmchwt_num_edges(self.h, m)

    def assemble(self, optsA, optsP, precond="S_INT"):
        pmchwt_assemble(self.h, optsA, optsP, precond)

    def get_block(self, op, medium, space, m=0, l=0):
        return pmchwt_get_block(self.h, op, medium, space, m, l)

    def get_entries(self, op, medium, space, m, l, rows, cols):
        return pmchwt_get_entries(self.h, op, medium, space, m, l, rows, cols)

    def get_mass(self, m=0):
        return pmchwt_get_mass(self.h, m)

    def rhs(self, dirs, pols):
        return pmchwt_rhs(self.h, dirs, pols)

    def apply(self, which, x):
        return pmchwt_apply(self.h, which, x)

    def solve(self, dirs, pols, opts, allow_not_converged=False):
        return pmchwt_solve(self.h, dirs, pols, opts, allow_not_converged)

    def apply_device(self, which, x_dev, nrhs, y_dev, stream=None):
        return pmchwt_apply_device(self.h, which, x_dev, nrhs, y_dev, stream)

    def solve_device(self, dirs, pols, opts, currents_dev, stream=None, allow_not_converged=False):
        return pmchwt_solve_device(self.h, dirs, pols, opts, currents_dev, stream, allow_not_converged)

    def far_field_device(self, currents_dev, nrhs, obs_dev, nobs, F_dev, stream=None):
        return pmchwt_far_field_device(self.h, currents_dev, nrhs, obs_dev, nobs, F_dev, stream)

    def far_field(self, currents, obs):
        return pmchwt_far_field(self.h, currents, obs)

    def far_field_noalloc(self, currents, obs):
        return pmchwt_far_field_noalloc(self.h, currents, obs)

    def near_field(self, currents, dirs, pols, points):
        return pmchwt_near_field(self.h, currents, dirs, pols, points)

    def cross_sections(self, currents, dirs, pols):
        return pmchwt_cross_sections(self.h, currents, dirs, pols)

    def profile(self):
        return pmchwt_get_profile(self.h)


# ---------------------------------------------------------------------------
# Serving (C ABI pmchwt_server_*)
# ---------------------------------------------------------------------------
def _result_dict(r):
    st = r.stats
    return {"status": r.status, "nrhs": r.nrhs, "n_unknowns": r.n_unknowns, "device_bytes": r.device_bytes,
            "ms_queued": r.ms_queued, "ms_total": r.ms_total, "iterations": st.iterations,
            "converged": bool(st.converged), "matvecs": st.matvecs, "rel_residual": st.rel_residual,
            "ir_steps": st.ir_steps, "restarts": st.restarts, "ms_solve": st.ms_solve}


def pmchwt_server_create(device, hbm_budget_bytes, max_live):
    h = _P()
    o = pmchwt_server_opts(int(hbm_budget_bytes), int(max_live))
    rc = _lib.pmchwt_server_create(ctypes.byref(h), device, ctypes.byref(o))
    if rc != OK:
        raise PmchwtError(rc, "pmchwt_server_create failed")
    return h


def pmchwt_server_submit(srv, meshes, eps, k_ext, dirs, pols, optsA, optsP, precond, solver):
    """meshes: [(verts, tris), ...]; eps: scalar or one per scatterer."""
    d, p = _waves(dirs, pols)
    M = len(meshes)
    vs = [_f64(v).reshape(-1, 3) for v, _ in meshes]
    ts = [np.ascontiguousarray(t, dtype=np.int32).reshape(-1, 3) for _, t in meshes]
    eps = np.broadcast_to(np.asarray(eps, dtype=np.complex128), (M,))
    vp = (ctypes.POINTER(ctypes.c_double) * M)(*[_ptr(v, _pd) for v in vs])
    tp = (ctypes.POINTER(ctypes.c_int32) * M)(*[_ptr(t, _pi32) for t in ts])
    nv = np.array([len(v) for v in vs], dtype=np.int32)
    nt = np.array([len(t) for t in ts], dtype=np.int32)
    ep = (pmchwt_complex * M)(*[pmchwt_complex(e.real, e.imag) for e in eps])
    pc = _c128(p).reshape(-1)
    req = pmchwt_request(M, ctypes.cast(vp, ctypes.POINTER(ctypes.POINTER(ctypes.c_double))), _ptr(nv, _pi32),
                         ctypes.cast(tp, ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))), _ptr(nt, _pi32),
                         ctypes.cast(ep, _pc), float(k_ext), len(d), _ptr(d, _pd), _ptr(pc, _pc),
                         optsA, optsP, PRECOND[precond] if isinstance(precond, str) else int(precond), solver)
    t = ctypes.c_uint64()
    rc = _lib.pmchwt_server_submit(srv, ctypes.byref(req), ctypes.byref(t))
    if rc != OK:
        raise PmchwtError(rc, "pmchwt_server_submit failed")
    return t.value


def pmchwt_server_poll(srv, ticket):
    r = pmchwt_result()
    _check(None, _lib.pmchwt_server_poll(srv, ticket, ctypes.byref(r)))
    return _result_dict(r)


def pmchwt_server_wait(srv, ticket, timeout_ms=-1.0):
    r = pmchwt_result()
    rc = _lib.pmchwt_server_wait(srv, ticket, float(timeout_ms), ctypes.byref(r))
    if rc not in (OK, RUNNING):
        raise PmchwtError(rc, "pmchwt_server_wait failed")
    return _result_dict(r)


def pmchwt_server_fetch(srv, ticket, nrhs, n_unknowns):
    cur = np.zeros(nrhs * n_unknowns, dtype=np.complex128)
    se, ss = np.zeros(nrhs), np.zeros(nrhs)
    _check(None, _lib.pmchwt_server_fetch(srv, ticket, _ptr(cur, _pc), _ptr(se, _pd), _ptr(ss, _pd)))
    return cur.reshape(nrhs, n_unknowns), se, ss


def pmchwt_server_cancel(srv, ticket):
    _check(None, _lib.pmchwt_server_cancel(srv, ticket))


def pmchwt_server_get_stats(srv):
    s = pmchwt_server_stats()
    _check(None, _lib.pmchwt_server_get_stats(srv, ctypes.byref(s)))
    return {f: getattr(s, f) for f, _ in pmchwt_server_stats._fields_}


def pmchwt_server_destroy(srv):
    _lib.pmchwt_server_destroy(srv)


class Server:
    """A serving loop on one GPU (see pmchwt_server_* in include/pmchwt.h)."""

    def __init__(self, device=0, hbm_budget_bytes=64 << 30, max_live=16):
        self.h = pmchwt_server_create(device, hbm_budget_bytes, max_live)

    def submit(self, meshes, eps, k_ext, dirs, pols, optsA, optsP, precond="S_INT", solver=None):
        solver = solver if solver is not None else solver_opts()
        return pmchwt_server_submit(self.h, meshes, eps, k_ext, dirs, pols, optsA, optsP, precond, solver)

    def poll(self, ticket):
        return pmchwt_server_poll(self.h, ticket)

    def wait(self, ticket, timeout_ms=-1.0):
        return pmchwt_server_wait(self.h, ticket, timeout_ms)

    def fetch(self, ticket):
        r = self.poll(ticket)
        return pmchwt_server_fetch(self.h, ticket, r["nrhs"], r["n_unknowns"])

    def cancel(self, ticket):
        pmchwt_server_cancel(self.h, ticket)

    def stats(self):
        return pmchwt_server_get_stats(self.h)

    def close(self):
        if self.h:
            pmchwt_server_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
