"""ctypes binding of the C ABI in include/cqm.h (argument marshalling only).

Function names match the C entry points.  Device buffers are passed as raw
integer addresses (for example torch tensors' data_ptr()); streams as raw
hipStream_t addresses (torch.cuda.current_stream().cuda_stream).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "CQM_OK", "CQM_EINVAL", "CQM_ENOMEM", "CQM_ENOCONV", "CQM_ENAN", "CQM_EDEVICE",
    "CQM_FP64_PLAIN", "CQM_MIXED_PLAIN", "CQM_MIXED_H2ACA", "CQM_FP64_H2ACA",
    "CQM_FORM_MATRIX_FREE", "CQM_FORM_DENSE", "CQM_BAND_FULL", "CQM_BAND_HALF", "KERNEL_CLASSES",
    "CQM_ARNOLDI_AUTO", "CQM_ARNOLDI_GROUP", "CQM_ARNOLDI_SPLIT",
    "CQM_PRECOND_NONE", "CQM_PRECOND_BLOCK_JACOBI",
    "CqmError", "cqm_options", "cqm_diag", "library_path", "load_library",
    "cqm_last_error", "cqm_default_options", "cqm_ctx_create", "cqm_ctx_destroy",
    "cqm_problem_create", "cqm_problem_destroy", "cqm_workspace_size", "cqm_set_workspace",
    "cqm_set_plane_wave", "cqm_set_dirichlet_samples", "cqm_solve", "cqm_solve_batch",
    "cqm_solve_marching", "CQM_FORMULATION_INDIRECT", "CQM_FORMULATION_DIRECT",
    "cqm_frequencies", "cqm_apply_V", "cqm_apply_V_noalloc", "cqm_apply_K", "cqm_apply_D",
    "cqm_near_entries", "cqm_operator_stats",
    "cqm_server_opts", "cqm_request", "cqm_server_stats_t", "cqm_server_default_options",
    "cqm_server_create", "cqm_server_submit", "cqm_server_poll", "cqm_server_drain",
    "cqm_server_stats", "cqm_server_destroy", "EXPORTED_SYMBOLS",
]

CQM_OK, CQM_EINVAL, CQM_ENOMEM, CQM_ENOCONV, CQM_ENAN, CQM_EDEVICE = 0, -1, -2, -3, -4, -5
CQM_FP64_PLAIN, CQM_MIXED_PLAIN, CQM_MIXED_H2ACA, CQM_FP64_H2ACA = 0, 1, 2, 3
CQM_FORM_MATRIX_FREE, CQM_FORM_DENSE = 0, 1
CQM_BAND_FULL, CQM_BAND_HALF = 0, 1
CQM_ARNOLDI_AUTO, CQM_ARNOLDI_GROUP, CQM_ARNOLDI_SPLIT = 0, 1, 2
CQM_PRECOND_NONE, CQM_PRECOND_BLOCK_JACOBI = 0, 1
CQM_FORMULATION_INDIRECT, CQM_FORMULATION_DIRECT = 0, 1
KERNEL_CLASSES = ["far32", "far64", "assemble", "gemv32", "gemv64", "near", "arnoldi", "other"]

EXPORTED_SYMBOLS = [
    "cqm_last_error", "cqm_default_options", "cqm_ctx_create", "cqm_ctx_destroy",
    "cqm_problem_create", "cqm_problem_destroy", "cqm_workspace_size", "cqm_set_workspace",
    "cqm_set_plane_wave", "cqm_set_dirichlet_samples", "cqm_solve", "cqm_solve_batch",
    "cqm_solve_marching", "cqm_frequencies", "cqm_apply_V", "cqm_apply_V_noalloc", "cqm_apply_K",
    "cqm_apply_D", "cqm_near_entries", "cqm_operator_stats",
    "cqm_server_default_options", "cqm_server_create", "cqm_server_submit", "cqm_server_poll",
    "cqm_server_drain", "cqm_server_stats", "cqm_server_destroy",
]


class CqmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class cqm_options(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32), ("form", ctypes.c_int32), ("rho", ctypes.c_double),
        ("gmres_restart", ctypes.c_int32), ("max_cycles", ctypes.c_int32),
        ("inner_tol", ctypes.c_double), ("outer_tol", ctypes.c_double),
        ("n_min", ctypes.c_int32), ("eta", ctypes.c_double), ("cheb_m", ctypes.c_int32),
        ("eps_aca", ctypes.c_double), ("aca_band", ctypes.c_int32), ("q_duffy", ctypes.c_int32),
        ("reuse_operator", ctypes.c_int32), ("profile", ctypes.c_int32),
        ("arnoldi_layout", ctypes.c_int32), ("autotune", ctypes.c_int32),
        ("graphs", ctypes.c_int32), ("precond", ctypes.c_int32), ("marching", ctypes.c_int32),
        ("cutoff_inner", ctypes.c_double), ("cutoff_outer", ctypes.c_double),
        ("refine_plain", ctypes.c_int32), ("formulation", ctypes.c_int32),
    ]


class cqm_diag(ctypes.Structure):
    _fields_ = [
        ("n_systems", ctypes.c_int32), ("cycles", ctypes.c_int32),
        ("total_iters", ctypes.c_int32), ("max_iters", ctypes.c_int32),
        ("max_rel_residual", ctypes.c_double), ("imag_ratio", ctypes.c_double),
        ("t_setup_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double),
        ("operator_bytes", ctypes.c_int64), ("converged", ctypes.c_int32),
        ("max_rank", ctypes.c_int32), ("mean_rank", ctypes.c_double),
        ("n_far_blocks", ctypes.c_int32), ("n_near_blocks", ctypes.c_int32),
        ("far_units", ctypes.c_int64), ("kernel_ms", ctypes.c_double * 8),
        ("kernel_calls", ctypes.c_int32 * 8), ("far_tile", ctypes.c_int32),
        ("far_waves", ctypes.c_int32), ("kernel_work", ctypes.c_double * 8),
        ("h2_plain_bytes", ctypes.c_int64), ("reserved", ctypes.c_int32 * 4),
    ]

    def as_dict(self):
        out = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        out["kernel_ms"] = list(self.kernel_ms)
        out["kernel_calls"] = list(self.kernel_calls)
        out["kernel_work"] = list(self.kernel_work)
        return out


class cqm_server_opts(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int32), ("cache_operators", ctypes.c_int32),
                ("large_lane", ctypes.c_int32), ("fail_after_cycles", ctypes.c_int32),
                ("large_cu_percent", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3),
                ("large_bytes", ctypes.c_int64), ("solver", cqm_options)]


class cqm_request(ctypes.Structure):
    _fields_ = [("vertices", ctypes.c_void_p), ("nv", ctypes.c_int64), ("tris", ctypes.c_void_p),
                ("M", ctypes.c_int64), ("N", ctypes.c_int32), ("T", ctypes.c_double),
                ("direction", ctypes.c_double * 3), ("sigma", ctypes.c_double),
                ("t0", ctypes.c_double), ("amplitude", ctypes.c_double)]


class cqm_server_stats_t(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "submitted", "completed", "rejected", "active", "queued", "peak_active", "arena_bytes",
        "peak_arena_bytes", "operators_built", "operator_cache_hits", "cycles")] + \
        [("lane_completed", ctypes.c_int64 * 2), ("arena_used", ctypes.c_int64),
         ("reserved", ctypes.c_int64 * 2)]

    def as_dict(self):
        out = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        out["lane_completed"] = list(self.lane_completed)
        return out


_lib = None


def library_path():
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libcqm.so")


def load_library():
    """Load lib/libcqm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise CqmError(CQM_EINVAL, f"{path} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(path)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "cqm_last_error": (ctypes.c_char_p, []),
        "cqm_default_options": (ctypes.c_int, [ctypes.POINTER(cqm_options)]),
        "cqm_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(P)]),
        "cqm_ctx_destroy": (ctypes.c_int, [P]),
        "cqm_problem_create": (ctypes.c_int, [P, P, I64, P, I64, I32, D,
                                              ctypes.POINTER(cqm_options), ctypes.POINTER(P)]),
        "cqm_problem_destroy": (ctypes.c_int, [P]),
        "cqm_workspace_size": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_size_t)]),
        "cqm_set_workspace": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "cqm_set_plane_wave": (ctypes.c_int, [P, ctypes.POINTER(D), D, D, D]),
        "cqm_set_dirichlet_samples": (ctypes.c_int, [P, P]),
        "cqm_solve": (ctypes.c_int, [P, P, ctypes.POINTER(cqm_diag), P]),
        "cqm_solve_marching": (ctypes.c_int, [P, P, ctypes.POINTER(cqm_diag), P]),
        "cqm_solve_batch": (ctypes.c_int, [ctypes.POINTER(P), I32, ctypes.POINTER(P),
                                           ctypes.POINTER(cqm_diag), P]),
        "cqm_frequencies": (ctypes.c_int, [I32, D, D, P, P]),
        "cqm_apply_V": (ctypes.c_int, [P, I32, I32, I32, P, P, P]),
        "cqm_apply_V_noalloc": (ctypes.c_int, [P, I32, I32, I32, P, P, P]),
        "cqm_apply_K": (ctypes.c_int, [P, I32, I32, I32, P, P, P]),
        "cqm_apply_D": (ctypes.c_int, [P, I32, I32, P, P, P]),
        "cqm_near_entries": (ctypes.c_int, [P, ctypes.POINTER(I64), P, P, P]),
        "cqm_operator_stats": (ctypes.c_int, [P, ctypes.POINTER(cqm_diag)]),
        "cqm_server_default_options": (ctypes.c_int, [ctypes.POINTER(cqm_server_opts)]),
        "cqm_server_create": (ctypes.c_int, [P, ctypes.c_size_t, ctypes.POINTER(cqm_server_opts),
                                             ctypes.POINTER(P)]),
        "cqm_server_submit": (ctypes.c_int, [P, ctypes.POINTER(cqm_request),
                                             ctypes.POINTER(ctypes.c_uint64)]),
        "cqm_server_poll": (ctypes.c_int, [P, ctypes.c_uint64, ctypes.POINTER(I32), P,
                                           ctypes.POINTER(cqm_diag), ctypes.POINTER(D)]),
        "cqm_server_drain": (ctypes.c_int, [P]),
        "cqm_server_stats": (ctypes.c_int, [P, ctypes.POINTER(cqm_server_stats_t)]),
        "cqm_server_destroy": (ctypes.c_int, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    _lib = L
    return L


def cqm_last_error():
    return load_library().cqm_last_error().decode()


def _check(rc, ok=(CQM_OK,)):
    if rc not in ok:
        raise CqmError(rc, cqm_last_error())
    return rc


def cqm_default_options(**overrides):
    o = cqm_options()
    _check(load_library().cqm_default_options(ctypes.byref(o)))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def cqm_ctx_create(device=0):
    h = ctypes.c_void_p()
    _check(load_library().cqm_ctx_create(device, ctypes.byref(h)))
    return h


def cqm_ctx_destroy(ctx):
    return _check(load_library().cqm_ctx_destroy(ctx))


def cqm_problem_create(ctx, vertices, tris, N, T, options=None):
    """vertices (nv,3) float64 and tris (M,3) int32 host arrays."""
    V = np.ascontiguousarray(vertices, dtype=np.float64)
    Tr = np.ascontiguousarray(tris, dtype=np.int32)
    h = ctypes.c_void_p()
    opt = options if options is not None else cqm_default_options()
    _check(load_library().cqm_problem_create(ctx, V.ctypes.data, V.shape[0], Tr.ctypes.data,
                                             Tr.shape[0], int(N), float(T), ctypes.byref(opt),
                                             ctypes.byref(h)))
    return h


def cqm_problem_destroy(p):
    return _check(load_library().cqm_problem_destroy(p))


def cqm_workspace_size(p):
    n = ctypes.c_size_t()
    _check(load_library().cqm_workspace_size(p, ctypes.byref(n)))
    return n.value


def cqm_set_workspace(p, dev_ptr, nbytes):
    return _check(load_library().cqm_set_workspace(p, ctypes.c_void_p(dev_ptr), nbytes))


def cqm_set_plane_wave(p, direction, sigma, t0, amplitude=1.0):
    d = (ctypes.c_double * 3)(*[float(x) for x in direction])
    return _check(load_library().cqm_set_plane_wave(p, d, sigma, t0, amplitude))


def cqm_set_dirichlet_samples(p, dev_ptr):
    return _check(load_library().cqm_set_dirichlet_samples(p, ctypes.c_void_p(dev_ptr)))


def cqm_solve_marching(p, q_out_ptr, stream=0):
    """Returns (rc, diag); rc is CQM_OK or CQM_ENOCONV, other codes raise."""
    d = cqm_diag()
    rc = load_library().cqm_solve_marching(p, ctypes.c_void_p(q_out_ptr), ctypes.byref(d),
                                           ctypes.c_void_p(stream))
    _check(rc, ok=(CQM_OK, CQM_ENOCONV))
    return rc, d


def cqm_solve(p, q_out_ptr, stream=0):
    """Returns (rc, diag); rc is CQM_OK or CQM_ENOCONV, other codes raise."""
    d = cqm_diag()
    rc = load_library().cqm_solve(p, ctypes.c_void_p(q_out_ptr), ctypes.byref(d),
                                  ctypes.c_void_p(stream))
    _check(rc, ok=(CQM_OK, CQM_ENOCONV))
    return rc, d


def cqm_solve_batch(problems, q_out_ptrs, stream=0):
    n = len(problems)
    arr = (ctypes.c_void_p * n)(*[p.value if isinstance(p, ctypes.c_void_p) else p for p in problems])
    outs = (ctypes.c_void_p * n)(*q_out_ptrs)
    diags = (cqm_diag * n)()
    rc = load_library().cqm_solve_batch(arr, n, outs, diags, ctypes.c_void_p(stream))
    _check(rc, ok=(CQM_OK, CQM_ENOCONV))
    return rc, list(diags)


def cqm_frequencies(N, T, rho=0.0):
    re = np.empty(N + 1)
    im = np.empty(N + 1)
    _check(load_library().cqm_frequencies(N, T, rho, re.ctypes.data, im.ctypes.data))
    return re + 1j * im


def cqm_apply_V(p, l0, nl, precision, x_ptr, y_ptr, stream=0):
    return _check(load_library().cqm_apply_V(p, l0, nl, precision, ctypes.c_void_p(x_ptr),
                                             ctypes.c_void_p(y_ptr), ctypes.c_void_p(stream)))


def cqm_apply_V_noalloc(p, l0, nl, precision, x_ptr, y_ptr, stream=0):
    return _check(load_library().cqm_apply_V_noalloc(p, l0, nl, precision, ctypes.c_void_p(x_ptr),
                                                     ctypes.c_void_p(y_ptr),
                                                     ctypes.c_void_p(stream)))


def cqm_apply_K(p, l0, nl, x_ptr, y_ptr, stream=0, adjoint=0):
    return _check(load_library().cqm_apply_K(p, l0, nl, int(adjoint), ctypes.c_void_p(x_ptr),
                                             ctypes.c_void_p(y_ptr), ctypes.c_void_p(stream)))


def cqm_apply_D(p, l0, nl, x_ptr, y_ptr, stream=0):
    return _check(load_library().cqm_apply_D(p, l0, nl, ctypes.c_void_p(x_ptr), ctypes.c_void_p(y_ptr),
                                             ctypes.c_void_p(stream)))


def cqm_near_entries(p, with_static=True):
    nnz = ctypes.c_int64()
    L = load_library()
    _check(L.cqm_near_entries(p, ctypes.byref(nnz), None, None, None))
    n = nnz.value
    stats = cqm_diag()
    _check(L.cqm_operator_stats(p, ctypes.byref(stats)))
    # row_ptr length is M+1; M is recovered from far_units bookkeeping-free call below
    rp = np.empty(_problem_M(p) + 1, dtype=np.int32)
    col = np.empty(n, dtype=np.int32)
    sv = np.empty(n, dtype=np.float64) if with_static else None
    _check(L.cqm_near_entries(p, ctypes.byref(nnz), rp.ctypes.data, col.ctypes.data,
                              sv.ctypes.data if with_static else None))
    return rp, col, sv


_M_of = {}


def _problem_M(p):
    return _M_of[p.value]


def cqm_operator_stats(p):
    d = cqm_diag()
    _check(load_library().cqm_operator_stats(p, ctypes.byref(d)))
    return d


_create = cqm_problem_create


def cqm_problem_create(ctx, vertices, tris, N, T, options=None):  # noqa: F811
    h = _create(ctx, vertices, tris, N, T, options)
    _M_of[h.value] = int(np.asarray(tris).shape[0])
    return h


def cqm_server_default_options(**solver):
    o = cqm_server_opts()
    _check(load_library().cqm_server_default_options(ctypes.byref(o)))
    for k, v in solver.items():
        if k in ("max_active", "cache_operators", "large_lane", "large_bytes", "fail_after_cycles"):
            setattr(o, k, v)
        else:
            setattr(o.solver, k, v)
    return o


def cqm_server_create(ctx, hbm_budget, opts=None):
    h = ctypes.c_void_p()
    o = opts if opts is not None else cqm_server_default_options()
    _check(load_library().cqm_server_create(ctx, int(hbm_budget), ctypes.byref(o), ctypes.byref(h)))
    return h


def cqm_server_submit(server, vertices, tris, N, T, direction=(1.0, 0.0, 0.0), sigma=0.25,
                      t0=1.5, amplitude=1.0):
    V = np.ascontiguousarray(vertices, dtype=np.float64)
    Tr = np.ascontiguousarray(tris, dtype=np.int32)
    r = cqm_request(V.ctypes.data, V.shape[0], Tr.ctypes.data, Tr.shape[0], int(N), float(T),
                    (ctypes.c_double * 3)(*[float(x) for x in direction]), float(sigma),
                    float(t0), float(amplitude))
    t = ctypes.c_uint64()
    _check(load_library().cqm_server_submit(server, ctypes.byref(r), ctypes.byref(t)))
    return t.value


def cqm_server_poll(server, ticket, out=None):
    """Returns (done, rc, diag, latency_ms); `out` (float64 numpy, (N+1)*M)
    receives the density when done == 1."""
    done = ctypes.c_int32()
    d = cqm_diag()
    lat = ctypes.c_double()
    ptr = out.ctypes.data if out is not None else None
    rc = load_library().cqm_server_poll(server, ctypes.c_uint64(ticket), ctypes.byref(done), ptr,
                                        ctypes.byref(d), ctypes.byref(lat))
    if done.value == 0:
        _check(rc)
    return done.value, rc, d, lat.value


def cqm_server_drain(server):
    return _check(load_library().cqm_server_drain(server))


def cqm_server_stats(server):
    s = cqm_server_stats_t()
    _check(load_library().cqm_server_stats(server, ctypes.byref(s)))
    return s


def cqm_server_destroy(server):
    return _check(load_library().cqm_server_destroy(server))
