"""ctypes binding of libbidomain.so -- argument marshalling only.

Every function here has the name of the C entry point it calls (see include/bidomain.h) and
does nothing but check and convert arguments: device vectors are torch CUDA tensors (their
data_ptr() is passed), host arrays are numpy arrays, streams default to torch's current
stream.  All computation runs in the HIP library; if it is not built, loading fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbidomain.so")

BD_OK, BD_E_NOT_CONVERGED = 0, 1
BD_E_INVALID, BD_E_NOMEM, BD_E_DEVICE, BD_E_BREAKDOWN, BD_E_NONFINITE, BD_E_BUDGET = -1, -2, -3, -4, -5, -6
BD_SA, BD_RS, BD_PMIS = 0, 1, 2
BD_CHEBYSHEV, BD_JACOBI = 0, 1
BD_F64, BD_F32 = 0, 1
BD_NULL_NONE, BD_NULL_CONSTANT = 0, 1
BD_PC_AMG, BD_PC_JACOBI, BD_PC_NONE = 0, 1, 2
BD_MIS_GREEDY, BD_MIS_LUBY = 0, 1
BD_OP_A, BD_OP_P, BD_OP_R, BD_OP_PRESMOOTH, BD_OP_VCYCLE, BD_OP_COARSE = range(6)
BD_MAT_AI, BD_MAT_AE, BD_MAT_AELL, BD_MAT_APAR = range(4)
BD_V, BD_UE, BD_W = range(3)
BD_MAX_LEVELS = 32

STATUS_NAMES = {0: "ok", 1: "not_converged", -1: "invalid", -2: "nomem", -3: "device", -4: "breakdown",
                -5: "nonfinite", -6: "budget"}


class bd_amg_opts(C.Structure):
    _fields_ = [("coarsening", C.c_int32), ("threshold", C.c_double), ("square_graph_levels", C.c_int32),
                ("prolong_smooths", C.c_int32), ("coarse_eq_limit", C.c_int32), ("max_levels", C.c_int32),
                ("smoother", C.c_int32), ("smoother_degree", C.c_int32), ("cheb_lo", C.c_double),
                ("cheb_hi", C.c_double), ("esteig_iters", C.c_int32), ("seed", C.c_uint64),
                ("vcycle_precision", C.c_int32), ("nullspace", C.c_int32), ("stagnation_ratio", C.c_double),
                ("coarse_dense_max", C.c_int32), ("galerkin_device", C.c_int32),
                ("diag_form", C.c_int32), ("preconditioner", C.c_int32), ("independent_set", C.c_int32),
                ("aggregate_device", C.c_int32), ("reorder", C.c_int32)]


class bd_csr(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int64), ("row_ptr", C.POINTER(C.c_int32)),
                ("col_idx", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double))]


class bd_solve_info(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("rel_residual_true", C.c_double), ("rel_residual_rec", C.c_double),
                ("seconds", C.c_double), ("status", C.c_int32)]


class bd_amg_stats(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("n", C.c_int64 * BD_MAX_LEVELS), ("nnz", C.c_int64 * BD_MAX_LEVELS),
                ("p_nnz", C.c_int64 * BD_MAX_LEVELS), ("lambda_", C.c_double * BD_MAX_LEVELS),
                ("coarse_mode", C.c_int32), ("operator_complexity", C.c_double), ("grid_complexity", C.c_double),
                ("device_bytes", C.c_int64), ("col_bytes", C.c_int32 * BD_MAX_LEVELS),
                ("tiles", C.c_int64 * BD_MAX_LEVELS), ("col_bytes_p", C.c_int32 * BD_MAX_LEVELS),
                ("col_bytes_r", C.c_int32 * BD_MAX_LEVELS), ("diags", C.c_int32 * BD_MAX_LEVELS),
                ("vcycle_precision", C.c_int32), ("renumbered", C.c_int32 * BD_MAX_LEVELS)]


class bd_slab(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("Lx", C.c_double), ("Ly", C.c_double),
                ("Lz", C.c_double), ("sig_il", C.c_double), ("sig_it", C.c_double), ("sig_el", C.c_double),
                ("sig_et", C.c_double), ("fiber_theta0", C.c_double), ("fiber_rotation", C.c_double),
                ("cm", C.c_double), ("dt", C.c_double), ("ap_k", C.c_double), ("ap_a", C.c_double),
                ("ap_eps0", C.c_double), ("ap_mu1", C.c_double), ("ap_mu2", C.c_double), ("ap_t_unit", C.c_double),
                ("ap_v_scale", C.c_double), ("ap_v_rest", C.c_double)]


class bd_ellipsoid(C.Structure):
    _fields_ = [("n_theta", C.c_int32), ("n_phi", C.c_int32), ("n_r", C.c_int32)] + \
        [(f, C.c_double) for f in ("a1", "a2", "b1", "b2", "c1", "c2", "theta_min", "theta_max", "phi_min",
                                   "phi_max", "sig_il", "sig_it", "sig_el", "sig_et", "fiber_endo", "fiber_epi",
                                   "cm", "dt", "ap_k", "ap_a", "ap_eps0", "ap_mu1", "ap_mu2", "ap_t_unit",
                                   "ap_v_scale", "ap_v_rest")]


class bd_step_info(C.Structure):
    _fields_ = [("steps", C.c_int32), ("it_par", C.c_int32), ("it_ell", C.c_int32), ("ms_memb", C.c_double),
                ("ms_par", C.c_double), ("ms_ell", C.c_double), ("rel_res_par", C.c_double),
                ("rel_res_ell", C.c_double), ("status", C.c_int32)]


class bd_case_result(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("status", C.c_int32), ("steps", C.c_int32), ("it_par", C.c_int32),
                ("it_ell", C.c_int32), ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_ready", C.c_double),
                ("t_done", C.c_double), ("max_rel_residual", C.c_double), ("device_bytes", C.c_int64)]


class bd_serve_stats(C.Structure):
    _fields_ = [("queued", C.c_int32), ("setting_up", C.c_int32), ("running", C.c_int32), ("done", C.c_int32),
                ("bytes_in_use", C.c_int64), ("budget", C.c_int64), ("rounds", C.c_int64), ("solves", C.c_int64),
                ("host_enqueue_s", C.c_double), ("host_wait_s", C.c_double), ("host_exit_s", C.c_double),
                ("max_batched", C.c_int64)]


_vp = C.c_void_p
_SIGS = {
    "bidomain_default_opts": (None, [C.POINTER(bd_amg_opts)]),
    "bidomain_amg_setup": (C.c_int, [C.POINTER(bd_csr), C.POINTER(bd_amg_opts), C.POINTER(C.c_double), _vp,
                                     C.POINTER(_vp)]),
    "bidomain_amg_build_host": (C.c_int, [C.POINTER(bd_csr), C.POINTER(bd_amg_opts), C.POINTER(_vp)]),
    "bidomain_pcg_solve": (C.c_int, [_vp, _vp, _vp, C.c_int, C.c_double, C.c_int, _vp, C.POINTER(bd_solve_info)]),
    "bidomain_pcg_solve_noalloc": (C.c_int, [_vp, _vp, _vp, C.c_int, C.c_double, C.c_int, _vp,
                                             C.POINTER(bd_solve_info)]),
    "bidomain_amg_info": (C.c_int, [_vp, C.POINTER(bd_amg_stats)]),
    "bidomain_amg_destroy": (None, [_vp]),
    "bidomain_amg_export": (C.c_int, [_vp, C.c_int, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_double)]),
    "bidomain_amg_apply": (C.c_int, [_vp, C.c_int, C.c_int, _vp, _vp, _vp]),
    "bidomain_slab_assemble": (C.c_int, [C.POINTER(bd_slab), C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "bidomain_sim_create": (C.c_int, [C.POINTER(bd_slab), C.POINTER(bd_amg_opts), C.POINTER(bd_amg_opts), _vp, _vp,
                                      C.c_double, _vp, C.POINTER(_vp)]),
    "bidomain_galerkin": (C.c_int, [C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_double), C.c_int, C.c_int64, C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "bidomain_ellipsoid_assemble": (C.c_int, [C.POINTER(bd_ellipsoid), C.c_int, C.POINTER(C.c_int32),
                                              C.POINTER(C.c_int32), C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "bidomain_ellipsoid_sim_create": (C.c_int, [C.POINTER(bd_ellipsoid), C.POINTER(bd_amg_opts),
                                                C.POINTER(bd_amg_opts), _vp, _vp, C.c_double, _vp, C.POINTER(_vp)]),
    "bidomain_step": (C.c_int, [_vp, C.c_int, C.c_double, _vp, C.POINTER(bd_step_info)]),
    "bidomain_sim_get": (C.c_int, [_vp, C.c_int, _vp, _vp]),
    "bidomain_sim_hierarchy": (_vp, [_vp, C.c_int]),
    "bidomain_sim_destroy": (None, [_vp]),
    "bidomain_profile_enable": (None, [C.c_int]),
    "bidomain_profile_read": (None, [C.POINTER(C.c_double), C.POINTER(C.c_int64), C.c_int]),
    "bidomain_serve_create": (C.c_int, [C.c_int64, C.c_int32, C.POINTER(bd_amg_opts), C.POINTER(bd_amg_opts),
                                        C.c_double, _vp, C.POINTER(_vp)]),
    "bidomain_serve_submit": (C.c_int, [_vp, C.POINTER(bd_slab), C.POINTER(C.c_double), C.c_int32,
                                        C.POINTER(C.c_uint64)]),
    "bidomain_serve_estimate": (C.c_int, [_vp, C.POINTER(bd_slab), C.POINTER(C.c_int64)]),
    "bidomain_serve_poll": (C.c_int, [_vp, C.POINTER(bd_case_result), C.c_int32, C.POINTER(C.c_int32)]),
    "bidomain_serve_fetch": (C.c_int, [_vp, C.c_uint64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "bidomain_serve_stats": (C.c_int, [_vp, C.POINTER(bd_serve_stats)]),
    "bidomain_serve_solve_latencies": (C.c_int, [_vp, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32)]),
    "bidomain_serve_destroy": (None, [_vp]),
    "bidomain_last_error": (C.c_char_p, []),
}

_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2311_13914_amd.build` "
                               "(there is no CPU fallback)")
        lib = C.CDLL(LIB_PATH)
        for name, (res, argt) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = argt
        _lib = lib
    return _lib


def exported_symbols():
    return list(_SIGS)


class BidomainError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = load().bidomain_last_error().decode()
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} ({msg})")


def _check(rc, where):
    if rc < 0:
        raise BidomainError(rc, where)
    return rc


def _stream(stream):
    if stream is None:
        import torch
        return _vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return _vp(stream)
    return _vp(stream.cuda_stream)


def _dev(t, dtype_name, n, name):
    import torch
    want = {"float64": torch.float64, "float32": torch.float32}[dtype_name]
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype != want or not t.is_contiguous() or t.numel() != n:
        raise ValueError(f"{name} must be a contiguous {dtype_name} tensor with {n} elements")
    return _vp(t.data_ptr())


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


# ---- options, slabs ---------------------------------------------------------------------
def bidomain_default_opts(**overrides) -> bd_amg_opts:
    o = bd_amg_opts()
    load().bidomain_default_opts(C.byref(o))
    names = {f[0] for f in bd_amg_opts._fields_}
    for k, v in overrides.items():
        if k not in names:
            raise KeyError(k)
        setattr(o, k, v)
    return o


def make_slab(case) -> bd_slab:
    """A bd_slab from any object with the slab attributes (nx, ny, nz, Lx, ..., cm, dt)."""
    return bd_slab(*(getattr(case, f[0]) for f in bd_slab._fields_))


def make_ellipsoid(case) -> bd_ellipsoid:
    """A bd_ellipsoid from any object with its attributes (n_theta, n_phi, n_r, a1, ..., ap_v_rest)."""
    return bd_ellipsoid(*(getattr(case, f[0]) for f in bd_ellipsoid._fields_))


# ---- hierarchy ---------------------------------------------------------------------------
class _Csr:
    def __init__(self, indptr, indices, data):
        self.rp, prp = _i32(indptr)
        self.ci, pci = _i32(indices)
        self.v, pv = _f64(data)
        n = self.rp.size - 1
        self.s = bd_csr(n, self.ci.size, prp, pci, pv)


def _as_csr(A):
    if hasattr(A, "indptr"):
        return _Csr(A.indptr, A.indices, A.data)
    indptr, indices, data = A
    return _Csr(indptr, indices, data)


def bidomain_amg_setup(A, opts: Optional[bd_amg_opts] = None, null_weights=None, stream=None):
    """A: scipy CSR matrix or (indptr, indices, data). Returns the handle (int)."""
    csr = _as_csr(A)
    o = opts or bidomain_default_opts()
    w = None
    pw = None
    if null_weights is not None:
        w, pw = _f64(null_weights)
        if w.size != csr.s.n:
            raise ValueError("null_weights must have n entries")
    out = _vp()
    _check(load().bidomain_amg_setup(C.byref(csr.s), C.byref(o), pw, _stream(stream), C.byref(out)),
           "bidomain_amg_setup")
    return out.value


def bidomain_amg_build_host(A, opts: Optional[bd_amg_opts] = None):
    csr = _as_csr(A)
    o = opts or bidomain_default_opts()
    out = _vp()
    _check(load().bidomain_amg_build_host(C.byref(csr.s), C.byref(o), C.byref(out)), "bidomain_amg_build_host")
    return out.value


def bidomain_amg_info(h) -> dict:
    s = bd_amg_stats()
    _check(load().bidomain_amg_info(_vp(h), C.byref(s)), "bidomain_amg_info")
    L = s.nlevels
    return dict(nlevels=L, n=list(s.n[:L]), nnz=list(s.nnz[:L]), p_nnz=list(s.p_nnz[:L]),
                lam=list(s.lambda_[:L]), coarse_mode=s.coarse_mode, operator_complexity=s.operator_complexity,
                grid_complexity=s.grid_complexity, device_bytes=s.device_bytes, col_bytes=list(s.col_bytes[:L]),
                tiles=list(s.tiles[:L]), col_bytes_p=list(s.col_bytes_p[:L]), col_bytes_r=list(s.col_bytes_r[:L]),
                diags=list(s.diags[:L]), vcycle_precision=s.vcycle_precision, renumbered=list(s.renumbered[:L]))


def bidomain_galerkin(A, P, on_device):
    """(R A P + (R A P)^T) / 2 with R = P^T (scipy CSR inputs; returns a scipy CSR matrix).
    on_device: False / 0 host, True / 1 the device's sparse product, 2 its dense MFMA product."""
    import scipy.sparse as sp
    A = sp.csr_matrix(A)
    P = sp.csr_matrix(P)
    n, nc = P.shape
    a = [np.ascontiguousarray(x, dt) for x, dt in ((A.indptr, np.int32), (A.indices, np.int32), (A.data, np.float64))]
    p = [np.ascontiguousarray(x, dt) for x, dt in ((P.indptr, np.int32), (P.indices, np.int32), (P.data, np.float64))]
    ip, dp = C.POINTER(C.c_int32), C.POINTER(C.c_double)
    args = [C.c_int32(n), C.c_int32(nc), a[0].ctypes.data_as(ip), a[1].ctypes.data_as(ip), a[2].ctypes.data_as(dp),
            p[0].ctypes.data_as(ip), p[1].ctypes.data_as(ip), p[2].ctypes.data_as(dp), int(on_device)]
    nnz = C.c_int64()
    rp = np.empty(nc + 1, np.int32)
    _check(load().bidomain_galerkin(*args, 0, rp.ctypes.data_as(ip), None, None, C.byref(nnz)), "bidomain_galerkin")
    ci = np.empty(nnz.value, np.int32)
    v = np.empty(nnz.value, np.float64)
    _check(load().bidomain_galerkin(*args, nnz.value, rp.ctypes.data_as(ip), ci.ctypes.data_as(ip),
                                    v.ctypes.data_as(dp), C.byref(nnz)), "bidomain_galerkin")
    return sp.csr_matrix((v, ci, rp), shape=(nc, nc))


def bidomain_amg_destroy(h):
    if h:
        load().bidomain_amg_destroy(_vp(h))


def bidomain_amg_export(h, level: int, which: int):
    """Level operator as (indptr, indices, data, shape): which 0 = A_k, 1 = P_k, 2 = R_k."""
    rows, cols, nnz = C.c_int32(), C.c_int32(), C.c_int64()
    lib = load()
    _check(lib.bidomain_amg_export(_vp(h), level, which, C.byref(rows), C.byref(cols), C.byref(nnz), None, None,
                                   None), "bidomain_amg_export")
    rp = np.empty(rows.value + 1, np.int32)
    ci = np.empty(nnz.value, np.int32)
    v = np.empty(nnz.value, np.float64)
    _check(lib.bidomain_amg_export(_vp(h), level, which, C.byref(rows), C.byref(cols), C.byref(nnz),
                                   rp.ctypes.data_as(C.POINTER(C.c_int32)), ci.ctypes.data_as(C.POINTER(C.c_int32)),
                                   v.ctypes.data_as(C.POINTER(C.c_double))), "bidomain_amg_export")
    return rp, ci, v, (rows.value, cols.value)


def bidomain_amg_apply(h, op: int, level: int, inp, out, stream=None):
    import torch
    for t, nm in ((inp, "in"), (out, "out")):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{nm} must be a contiguous CUDA tensor")
    info = bidomain_amg_info(h)
    nl = info["nlevels"]
    if not 0 <= level < nl:
        raise ValueError("level out of range")
    sizes = {BD_OP_A: (level, level), BD_OP_P: (level + 1, level), BD_OP_R: (level, level + 1),
             BD_OP_PRESMOOTH: (level, level), BD_OP_VCYCLE: (level, level), BD_OP_COARSE: (nl - 1, nl - 1)}
    if op not in sizes:
        raise ValueError("unknown op")
    li, lo = sizes[op]
    if max(li, lo) >= nl:
        raise ValueError("the coarsest level has no transfer operators")
    want = torch.float32 if info["vcycle_precision"] == BD_F32 else torch.float64
    if inp.dtype != want or out.dtype != want:
        raise ValueError(f"in and out must be {want} tensors: the hierarchy's V-cycle precision")
    if inp.numel() != info["n"][li] or out.numel() != info["n"][lo]:
        raise ValueError("vector sizes do not match the level")
    _check(load().bidomain_amg_apply(_vp(h), op, level, _vp(inp.data_ptr()), _vp(out.data_ptr()), _stream(stream)),
           "bidomain_amg_apply")


def bidomain_pcg_solve(h, b, x, x_is_guess: bool, rtol: float = 1e-8, maxit: int = 500, stream=None):
    """b, x: float64 CUDA tensors of n entries. Returns (status, info dict)."""
    return _solve("bidomain_pcg_solve", h, b, x, x_is_guess, rtol, maxit, stream)


def bidomain_pcg_solve_noalloc(h, b, x, x_is_guess: bool, rtol: float = 1e-8, maxit: int = 500, stream=None):
    """As bidomain_pcg_solve, with the solve state in the library's static device array."""
    return _solve("bidomain_pcg_solve_noalloc", h, b, x, x_is_guess, rtol, maxit, stream)


def _solve(name, h, b, x, x_is_guess, rtol, maxit, stream):
    n = bidomain_amg_info(h)["n"][0]
    pb = _dev(b, "float64", n, "b")
    px = _dev(x, "float64", n, "x")
    inf = bd_solve_info()
    rc = getattr(load(), name)(_vp(h), pb, px, int(bool(x_is_guess)), float(rtol), int(maxit), _stream(stream),
                               C.byref(inf))
    if rc < 0 and rc not in (BD_E_BREAKDOWN, BD_E_NONFINITE):
        raise BidomainError(rc, name)
    return rc, dict(iterations=inf.iterations, rel_residual_true=inf.rel_residual_true,
                    rel_residual_rec=inf.rel_residual_rec, seconds=inf.seconds, status=inf.status)


# ---- slab and simulation ------------------------------------------------------------------
def bidomain_slab_assemble(case, which: int):
    s = make_slab(case)
    n = (s.nx + 1) * (s.ny + 1) * (s.nz + 1)
    nnz = (3 * s.nx + 1) * (3 * s.ny + 1) * (3 * s.nz + 1)
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    v = np.empty(nnz, np.float64)
    m = np.empty(n, np.float64)
    _check(load().bidomain_slab_assemble(C.byref(s), which, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                                         ci.ctypes.data_as(C.POINTER(C.c_int32)),
                                         v.ctypes.data_as(C.POINTER(C.c_double)),
                                         m.ctypes.data_as(C.POINTER(C.c_double))), "bidomain_slab_assemble")
    return rp, ci, v, m


def bidomain_ellipsoid_assemble(case, which: int):
    e = make_ellipsoid(case)
    n = e.n_theta * (e.n_phi + 1) * (e.n_r + 1)
    nnz = 3 * e.n_theta * (3 * e.n_phi + 1) * (3 * e.n_r + 1)
    rp = np.empty(n + 1, np.int32)
    ci = np.empty(nnz, np.int32)
    v = np.empty(nnz, np.float64)
    m = np.empty(n, np.float64)
    _check(load().bidomain_ellipsoid_assemble(C.byref(e), which, rp.ctypes.data_as(C.POINTER(C.c_int32)),
                                              ci.ctypes.data_as(C.POINTER(C.c_int32)),
                                              v.ctypes.data_as(C.POINTER(C.c_double)),
                                              m.ctypes.data_as(C.POINTER(C.c_double))),
           "bidomain_ellipsoid_assemble")
    return rp, ci, v, m


def bidomain_sim_create(case, v0, w0=None, rtol: float = 1e-8, ell_opts=None, par_opts=None, stream=None):
    """A simulation of a slab case, or of an ellipsoid case (a case with n_theta)."""
    ellipsoid = hasattr(case, "n_theta")
    s = make_ellipsoid(case) if ellipsoid else make_slab(case)
    n = case.n_theta * (case.n_phi + 1) * (case.n_r + 1) if ellipsoid else (s.nx + 1) * (s.ny + 1) * (s.nz + 1)
    pv = _dev(v0, "float64", n, "v0")
    pw = _dev(w0, "float64", n, "w0") if w0 is not None else None
    out = _vp()
    fn = load().bidomain_ellipsoid_sim_create if ellipsoid else load().bidomain_sim_create
    _check(fn(C.byref(s), C.byref(ell_opts) if ell_opts else None, C.byref(par_opts) if par_opts else None, pv, pw,
              float(rtol), _stream(stream), C.byref(out)),
           "bidomain_ellipsoid_sim_create" if ellipsoid else "bidomain_sim_create")
    return out.value


def bidomain_step(sim, nsteps: int, rtol: float = 1e-8, stream=None):
    inf = bd_step_info()
    rc = load().bidomain_step(_vp(sim), int(nsteps), float(rtol), _stream(stream), C.byref(inf))
    if rc < 0 and rc not in (BD_E_BREAKDOWN, BD_E_NONFINITE):
        raise BidomainError(rc, "bidomain_step")
    return rc, {f[0]: getattr(inf, f[0]) for f in bd_step_info._fields_}


def bidomain_sim_get(sim, field: int, out, stream=None):
    h = bidomain_sim_hierarchy(sim, 0)
    n = bidomain_amg_info(h)["n"][0]
    _check(load().bidomain_sim_get(_vp(sim), field, _dev(out, "float64", n, "out"), _stream(stream)),
           "bidomain_sim_get")


def bidomain_sim_hierarchy(sim, which: int):
    return load().bidomain_sim_hierarchy(_vp(sim), which)


def bidomain_sim_destroy(sim):
    if sim:
        load().bidomain_sim_destroy(_vp(sim))


def bidomain_profile_enable(on: bool):
    load().bidomain_profile_enable(int(bool(on)))


def bidomain_profile_read(reset: bool = False):
    ms, cnt = C.c_double(), C.c_int64()
    load().bidomain_profile_read(C.byref(ms), C.byref(cnt), int(bool(reset)))
    return ms.value, cnt.value


def bidomain_last_error() -> str:
    return load().bidomain_last_error().decode()


# ---- serving -------------------------------------------------------------------------------
def bidomain_serve_create(budget_bytes: int, max_slots: int, ell_opts=None, par_opts=None, rtol: float = 1e-8,
                          stream=None):
    out = _vp()
    _check(load().bidomain_serve_create(int(budget_bytes), int(max_slots), C.byref(ell_opts) if ell_opts else None,
                                        C.byref(par_opts) if par_opts else None, float(rtol), _stream(stream),
                                        C.byref(out)), "bidomain_serve_create")
    return out.value


def bidomain_serve_submit(srv, case, v0, nsteps: int) -> int:
    """v0: host array of n doubles. Returns the ticket; raises BidomainError (BD_E_BUDGET) if the
    case can never fit the budget."""
    s = make_slab(case)
    n = (s.nx + 1) * (s.ny + 1) * (s.nz + 1)
    v, pv = _f64(v0)
    if v.size != n:
        raise ValueError("v0 must have n entries")
    t = C.c_uint64()
    _check(load().bidomain_serve_submit(_vp(srv), C.byref(s), pv, int(nsteps), C.byref(t)), "bidomain_serve_submit")
    return t.value


def bidomain_serve_estimate(srv, case) -> int:
    s = make_slab(case)
    b = C.c_int64()
    _check(load().bidomain_serve_estimate(_vp(srv), C.byref(s), C.byref(b)), "bidomain_serve_estimate")
    return b.value


def bidomain_serve_poll(srv, max_results: int = 64):
    res = (bd_case_result * max_results)()
    cnt = C.c_int32()
    _check(load().bidomain_serve_poll(_vp(srv), res, int(max_results), C.byref(cnt)), "bidomain_serve_poll")
    return [{f[0]: getattr(res[i], f[0]) for f in bd_case_result._fields_} for i in range(cnt.value)]


def bidomain_serve_fetch(srv, ticket: int, n: int):
    v = np.empty(n, np.float64)
    ue = np.empty(n, np.float64)
    _check(load().bidomain_serve_fetch(_vp(srv), C.c_uint64(ticket), v.ctypes.data_as(C.POINTER(C.c_double)),
                                       ue.ctypes.data_as(C.POINTER(C.c_double))), "bidomain_serve_fetch")
    return v, ue


def bidomain_serve_stats(srv) -> dict:
    st = bd_serve_stats()
    _check(load().bidomain_serve_stats(_vp(srv), C.byref(st)), "bidomain_serve_stats")
    return {f[0]: getattr(st, f[0]) for f in bd_serve_stats._fields_}


def bidomain_serve_solve_latencies(srv):
    cnt = C.c_int32()
    _check(load().bidomain_serve_solve_latencies(_vp(srv), None, 0, C.byref(cnt)), "bidomain_serve_solve_latencies")
    out = np.empty(cnt.value, np.float64)
    _check(load().bidomain_serve_solve_latencies(_vp(srv), out.ctypes.data_as(C.POINTER(C.c_double)), cnt.value,
                                                 C.byref(cnt)), "bidomain_serve_solve_latencies")
    return out


def bidomain_serve_destroy(srv):
    if srv:
        load().bidomain_serve_destroy(_vp(srv))
