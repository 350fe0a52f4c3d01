"""Thin Python binding of libzolo.so (the MI355X Zolotarev spectrum-filter eigensolver).

Argument marshalling only: every step of the method runs in the library's HIP
kernels and host C++ code.  PyTorch supplies device memory (tensors on the
GPU, passed by ``data_ptr()``) and the current HIP stream.  The names follow
``include/zolo.h``; the library raises if it has not been built.
"""
from __future__ import annotations

import ctypes
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libzolo.so")

ZOLO_OK, ZOLO_EINVAL, ZOLO_ENOTHERM, ZOLO_ENOMEM, ZOLO_ENOCONV = 0, 1, 2, 3, 4
ZOLO_EGAP, ZOLO_ESUBSPACE, ZOLO_EDEVICE, ZOLO_EBREAKDOWN, ZOLO_ETIMEOUT = 5, 6, 7, 8, 9
ZOLO_REAL64, ZOLO_COMPLEX128 = 0, 1
ZOLO_PREC_FP64, ZOLO_PREC_MIXED = 0, 1
ZOLO_MAX_R = 16
ZOLO_FILTER_HYBRID, ZOLO_FILTER_ZOLO, ZOLO_FILTER_TRAPEZOID, ZOLO_FILTER_GAUSS = 0, 1, 2, 3
STATUS_NAMES = {0: "ZOLO_OK", 1: "ZOLO_EINVAL", 2: "ZOLO_ENOTHERM", 3: "ZOLO_ENOMEM", 4: "ZOLO_ENOCONV",
                5: "ZOLO_EGAP", 6: "ZOLO_ESUBSPACE", 7: "ZOLO_EDEVICE", 8: "ZOLO_EBREAKDOWN",
                9: "ZOLO_ETIMEOUT"}

_R = ZOLO_MAX_R
_d = ctypes.c_double
_i = ctypes.c_int
_i64 = ctypes.c_int64
_vp = ctypes.c_void_p


class zolo_filter_coeffs(ctypes.Structure):
    _fields_ = [("r1", _i), ("r2", _i), ("a_minus", _d), ("a_plus", _d), ("b_minus", _d), ("b_plus", _d),
                ("l1", _d), ("l2", _d), ("alpha", _d), ("beta", _d), ("gamma", _d), ("M_hat", _d), ("c0", _d),
                ("delta1", _d), ("sigma_hat_re", _d * _R), ("sigma_hat_im", _d * _R), ("w_hat_re", _d * _R),
                ("w_hat_im", _d * _R), ("a_hat", _d * _R), ("c_hat", _d * _R), ("M", _d), ("a", _d * _R),
                ("c", _d * _R), ("delta_S", _d), ("delta0", _d), ("kind", _i)]


class zolo_opts(ctypes.Structure):
    _fields_ = [("a_minus", _d), ("a_plus", _d), ("b_minus", _d), ("b_plus", _d), ("r1", _i), ("r2", _i),
                ("filter_eps", _d), ("n_ss", _i), ("max_subspace_iter", _i), ("max_gmres_iter", _i),
                ("tol_resid", _d), ("tol_gmres", _d), ("precision", _i), ("seed", ctypes.c_uint64),
                ("max_refine", _i), ("tol_refine", _d), ("block_cols", _i), ("filter_kind", _i),
                ("gmres_restart", _i), ("reuse_subspace", _i)]


class zolo_stats(ctypes.Structure):
    _fields_ = [("n_iter", _i), ("n_gmres_total", _i), ("n_gmres_last", _i), ("n_solv", ctypes.c_longlong),
                ("n_refine", ctypes.c_longlong), ("refine_sweeps_max", _i), ("refine_missed", _i),
                ("refine_worst", _d), ("n_found", _i), ("max_resid", _d), ("e_lambda_x", _d),
                ("b_orth", _d), ("t_plan", _d), ("t_symbolic", _d), ("t_factor", _d), ("t_iter", _d),
                ("t_total", _d), ("gmres_resid", _d), ("norm_a", _d), ("norm_b", _d), ("r1", _i), ("r2", _i),
                ("l1", _d), ("l2", _d), ("delta0", _d), ("factor_bytes", ctypes.c_longlong),
                ("nnz_l", ctypes.c_longlong), ("factor_flops", _d), ("inertia_count", ctypes.c_longlong),
                ("t_gaps", _d), ("a_minus", _d), ("a_plus", _d), ("b_minus", _d), ("b_plus", _d),
                ("factors_reused", _i), ("n_restart", _i), ("precision_fallback", _i), ("subspace_reused", _i)]


class zolo_kernel_profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_longlong), ("ms", _d), ("flops", _d), ("bytes", _d)]


PROF_CLASSES = ["spmm", "gemm_factor", "gemm_solve", "gemm_krylov", "front_other", "solve_gather", "hls", "rr",
                "elemwise"]


class zolo_query_info(ctypes.Structure):
    _fields_ = [("t_submit", _d), ("t_start", _d), ("t_end", _d), ("batch", _i), ("est_bytes", ctypes.c_longlong),
                ("done", _i)]


class zolo_server_info(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_longlong), ("running_bytes", ctypes.c_longlong),
                ("resident_factors", _i), ("resident_bytes", ctypes.c_longlong),
                ("factor_hits", ctypes.c_longlong), ("factor_misses", ctypes.c_longlong), ("queued", _i),
                ("subspace_hits", ctypes.c_longlong), ("resident_subspaces", _i)]


class zolo_filter_stats(ctypes.Structure):
    _fields_ = [("n_gmres", _i), ("worst_resid", _d), ("breakdown", _i), ("restarts", _i)]


def struct_dict(s) -> dict:
    out = {}
    for name, _ in s._fields_:
        v = getattr(s, name)
        out[name] = list(v) if hasattr(v, "__len__") else v
    return out


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "zolo_last_error": (ctypes.c_char_p, []),
    "zolo_version": (ctypes.c_char_p, []),
    "zolo_opts_default": (_i, [ctypes.POINTER(zolo_opts)]),
    "zolo_ctx_create": (_i, [_i, ctypes.POINTER(_vp)]),
    "zolo_ctx_destroy": (None, [_vp]),
    "zolo_ctx_set_hbm_budget": (_i, [_vp, ctypes.c_size_t]),
    "zolo_ctx_hbm_in_use": (_i, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "zolo_pencil_create": (_i, [_vp, _i64, _vp, _vp, _vp, _vp, _i, _vp, _i, ctypes.POINTER(_vp)]),
    "zolo_pencil_free": (None, [_vp]),
    "zolo_pencil_info": (_i, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                              ctypes.POINTER(_d), ctypes.POINTER(_i64)]),
    "zolo_pencil_perm": (_i, [_vp, _vp]),
    "zolo_pencil_memory": (_i, [_vp, _vp]),
    "zolo_pencil_flops": (_i, [_vp, _vp]),
    "zolo_symbolic": (_i, [_i64, _vp, _vp, _vp, _i, _vp, _vp]),
    "zolo_filter_plan": (_i, [_d, _d, _d, _d, _i, _i, _d, ctypes.POINTER(zolo_filter_coeffs)]),
    "zolo_filter_plan_kind": (_i, [_i, _d, _d, _d, _d, _d, _d, _i, _d, ctypes.POINTER(zolo_filter_coeffs)]),
    "zolo_factor": (_i, [_vp, _vp, ctypes.POINTER(zolo_filter_coeffs), _i, _vp, ctypes.POINTER(_vp)]),
    "zolo_factors_free": (None, [_vp]),
    "zolo_inertia": (_i, [_vp, _vp, _vp, _i, _vp, _vp]),
    "zolo_spmm": (_i, [_vp, _i, _vp, _i64, _i, _vp, _i64, _vp]),
    "zolo_residuals": (_i, [_vp, _vp, _i64, _i, _vp, _vp, _vp]),
    "zolo_residuals_noalloc": (_i, [_vp, _vp, _i64, _i, _vp, _vp, _vp]),
    "zolo_pole_solve": (_i, [_vp, _i, _vp, _i64, _i, _vp, _i64, _vp]),
    "zolo_apply_G": (_i, [_vp, _vp, _i64, _i, _vp, _i64, _vp]),
    "zolo_filter_apply": (_i, [_vp, _vp, _i64, _i, _vp, _i64, _d, _i, _i, ctypes.POINTER(zolo_filter_stats), _vp]),
    "zolo_solve": (_i, [_vp, _vp, _d, _d, _i, ctypes.POINTER(zolo_opts), _vp, _vp, ctypes.POINTER(_vp)]),
    "zolo_slice": (_i, [_vp, _vp, _d, _d, _i, ctypes.POINTER(zolo_opts), _vp, ctypes.POINTER(_vp)]),
    "zolo_result_count": (_i64, [_vp]),
    "zolo_result_eigenvalues": (ctypes.POINTER(_d), [_vp]),
    "zolo_result_copy_vectors": (_i, [_vp, _vp, _i64, _vp]),
    "zolo_result_copy_vectors_host": (_i, [_vp, _vp, _i64]),
    "zolo_result_device_vectors": (_vp, [_vp, ctypes.POINTER(_i64)]),
    "zolo_result_stats": (_i, [_vp, ctypes.POINTER(zolo_stats)]),
    "zolo_result_free": (None, [_vp]),
    "zolo_profile_enable": (_i, [_i]),
    "zolo_profile_query": (_i, [_i, ctypes.POINTER(zolo_kernel_profile)]),
    "zolo_server_create": (_i, [_vp, _i, ctypes.c_size_t, ctypes.POINTER(_vp)]),
    "zolo_submit": (_i, [_vp, _vp, _d, _d, _i, ctypes.POINTER(zolo_opts), _vp, ctypes.POINTER(_vp)]),
    "zolo_wait": (_i, [_vp, _i, ctypes.POINTER(_vp)]),
    "zolo_query_get_info": (_i, [_vp, ctypes.POINTER(zolo_query_info)]),
    "zolo_query_free": (None, [_vp]),
    "zolo_server_get_info": (_i, [_vp, ctypes.POINTER(zolo_server_info)]),
    "zolo_server_drop_pencil": (_i, [_vp, _vp]),
    "zolo_server_destroy": (None, [_vp]),
}


class ZoloError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def lib():
    """Load libzolo.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1701_08935_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, allow=()):
    if rc != ZOLO_OK and rc not in allow:
        raise ZoloError(rc, lib().zolo_last_error().decode())
    return rc


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
def zolo_filter_plan(a_minus, a_plus, b_minus, b_plus, r1, r2=0, eps=1e-10) -> zolo_filter_coeffs:
    co = zolo_filter_coeffs()
    _check(lib().zolo_filter_plan(float(a_minus), float(a_plus), float(b_minus), float(b_plus), int(r1), int(r2),
                                  float(eps), ctypes.byref(co)))
    return co


def zolo_filter_plan_kind(kind, a, b, a_minus=float("nan"), a_plus=float("nan"), b_minus=float("nan"),
                          b_plus=float("nan"), r=2, eps=1e-10) -> zolo_filter_coeffs:
    co = zolo_filter_coeffs()
    _check(lib().zolo_filter_plan_kind(int(kind), float(a), float(b), float(a_minus), float(a_plus), float(b_minus),
                                       float(b_plus), int(r), float(eps), ctypes.byref(co)))
    return co


def zolo_opts_default() -> zolo_opts:
    o = zolo_opts()
    _check(lib().zolo_opts_default(ctypes.byref(o)))
    return o


def zolo_symbolic(rowptr, colind, grid=None, leaf_size=0):
    import numpy as np

    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    colind = np.ascontiguousarray(colind, dtype=np.int32)
    n = rowptr.shape[0] - 1
    perm = np.empty(n, dtype=np.int32)
    info = np.empty(8, dtype=np.float64)
    g = None if grid is None else np.ascontiguousarray(grid, dtype=np.int32)
    _check(lib().zolo_symbolic(n, _np_ptr(rowptr), _np_ptr(colind), None if g is None else _np_ptr(g),
                               int(leaf_size), _np_ptr(perm), _np_ptr(info)))
    keys = ["fronts", "levels", "panel_entries", "inv_entries", "update_entries", "max_front", "struct_entries",
            "flops"]
    return perm, dict(zip(keys, info.tolist()))


class Context:
    def __init__(self, device: int = 0):
        h = _vp()
        _check(lib().zolo_ctx_create(int(device), ctypes.byref(h)))
        self.h = h
        self.device = device

    def set_hbm_budget(self, nbytes: int):
        """zolo_ctx_set_hbm_budget: device-memory budget of the library on this device (0 = none)."""
        _check(lib().zolo_ctx_set_hbm_budget(self.h, int(nbytes)))

    def hbm_in_use(self) -> int:
        v = ctypes.c_size_t()
        _check(lib().zolo_ctx_hbm_in_use(self.h, ctypes.byref(v)))
        return v.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.zolo_ctx_destroy(self.h)
            self.h = None


class Pencil:
    """zolo_pencil_create on host CSR arrays (numpy)."""

    def __init__(self, ctx: Context, rowptr, colind, a_vals, b_vals, grid=None, leaf_size=0):
        import numpy as np

        self.ctx = ctx
        self._rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        self._colind = np.ascontiguousarray(colind, dtype=np.int32)
        self.cplx = np.iscomplexobj(a_vals) or np.iscomplexobj(b_vals)
        vt = np.complex128 if self.cplx else np.float64
        self._a = np.ascontiguousarray(a_vals, dtype=vt)
        self._b = np.ascontiguousarray(b_vals, dtype=vt)
        self.n = self._rowptr.shape[0] - 1
        g = None if grid is None else np.ascontiguousarray(grid, dtype=np.int32)
        h = _vp()
        _check(lib().zolo_pencil_create(ctx.h, self.n, _np_ptr(self._rowptr), _np_ptr(self._colind), _np_ptr(self._a),
                                        _np_ptr(self._b), ZOLO_COMPLEX128 if self.cplx else ZOLO_REAL64,
                                        None if g is None else _np_ptr(g), int(leaf_size), ctypes.byref(h)))
        self.h = h

    @classmethod
    def from_grid(cls, ctx, gp, leaf_size=0, use_grid=True):
        return cls(ctx, gp.rowptr, gp.colind, gp.a_vals, gp.b_vals, gp.grid if use_grid else None, leaf_size)

    def info(self):
        nf, nl, nnz, mf = _i64(), _i64(), _i64(), _i64()
        fl = _d()
        _check(lib().zolo_pencil_info(self.h, ctypes.byref(nf), ctypes.byref(nl), ctypes.byref(nnz), ctypes.byref(fl),
                                      ctypes.byref(mf)))
        return {"fronts": nf.value, "levels": nl.value, "nnz_l": nnz.value, "flops": fl.value, "max_front": mf.value}

    def flops(self):
        """Algorithmic flops of one pole (zolo_pencil_flops)."""
        import numpy as np

        out = np.zeros(3, dtype=np.float64)
        _check(lib().zolo_pencil_flops(self.h, _np_ptr(out)))
        return dict(zip(["elimination", "with_inverses", "solve_per_column"], out.tolist()))

    def memory(self):
        """Factor-side entry counts of one pole (zolo_pencil_memory)."""
        import numpy as np

        out = np.zeros(6, dtype=np.int64)
        _check(lib().zolo_pencil_memory(self.h, _np_ptr(out)))
        return dict(zip(["panels", "inverses", "update_pool", "update_all", "inv_scratch", "conv_scratch"],
                        out.tolist()))

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.zolo_pencil_free(self.h)
            self.h = None


class Factors:
    """zolo_factor: LDL^T of A - sigma_hat_j B for j = 1..r1."""

    def __init__(self, ctx: Context, pencil: Pencil, coeffs: zolo_filter_coeffs, precision=ZOLO_PREC_FP64):
        h = _vp()
        self.pencil = pencil
        self.coeffs = coeffs
        _check(lib().zolo_factor(ctx.h, pencil.h, ctypes.byref(coeffs), int(precision), _stream(), ctypes.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.zolo_factors_free(self.h)
            self.h = None


def zolo_inertia(ctx: Context, pencil: Pencil, sigmas):
    """Number of eigenvalues of the pencil below each real shift (device LDL^T inertia)."""
    import numpy as np

    s = np.ascontiguousarray(sigmas, dtype=np.float64)
    out = np.zeros(s.shape[0], dtype=np.int64)
    _check(lib().zolo_inertia(ctx.h, pencil.h, _np_ptr(s), int(s.shape[0]), _np_ptr(out), _stream()))
    return out


def zolo_spmm(pencil: Pencil, which: int, X):
    import torch

    Y = torch.empty_like(X)
    _check(lib().zolo_spmm(pencil.h, int(which), _ptr(X), X.stride(0), X.shape[1], _ptr(Y), Y.stride(0), _stream()))
    return Y


def zolo_residuals(pencil: Pencil, X, lam):
    """Per-column ||A x - lam B x|| / ((||A||_inf + |lam| ||B||_inf) ||x||) on the device
    (X: N x k tensor of the pencil's scalar type, lam: k float64 tensor on the same device)."""
    import torch

    out = torch.empty(X.shape[1], dtype=torch.float64, device=X.device)
    _check(lib().zolo_residuals(pencil.h, _ptr(X), X.stride(0), X.shape[1], _ptr(lam), _ptr(out), _stream()))
    return out


def zolo_residuals_noalloc(pencil: Pencil, X, lam, out):
    """zolo_residuals into a caller-provided `out` (k float64 on the device) through the
    entry point that allocates nothing (the library's static scratch)."""
    _check(lib().zolo_residuals_noalloc(pencil.h, _ptr(X), X.stride(0), X.shape[1], _ptr(lam), _ptr(out), _stream()))
    return out


def zolo_pole_solve(f: Factors, j: int, T):
    import torch

    X = torch.empty(T.shape, dtype=torch.complex128, device=T.device)
    _check(lib().zolo_pole_solve(f.h, int(j), _ptr(T), T.stride(0), T.shape[1], _ptr(X), X.stride(0), _stream()))
    return X


def zolo_apply_G(f: Factors, V):
    import torch

    W = torch.empty_like(V)
    _check(lib().zolo_apply_G(f.h, _ptr(V), V.stride(0), V.shape[1], _ptr(W), W.stride(0), _stream()))
    return W


def zolo_filter_apply(f: Factors, V, tol=1e-10, max_iter=60, restart=0, allow_noconv=False):
    import torch

    Y = torch.empty_like(V)
    st = zolo_filter_stats()
    _check(lib().zolo_filter_apply(f.h, _ptr(V), V.stride(0), V.shape[1], _ptr(Y), Y.stride(0), float(tol),
                                   int(max_iter), int(restart), ctypes.byref(st), _stream()),
           allow=(ZOLO_ENOCONV,) if allow_noconv else ())
    return Y, struct_dict(st)


def zolo_slice(ctx: Context, pencil: Pencil, lo, hi, n_slices, opts: zolo_opts = None, allow=(ZOLO_ENOCONV,)):
    """Spectrum slicing: (eigenvalues, vectors N x count on the device, stats, status) of (lo, hi)."""
    import torch

    if opts is None:
        opts = zolo_opts_default()
    h = _vp()
    rc = lib().zolo_slice(ctx.h, pencil.h, float(lo), float(hi), int(n_slices), ctypes.byref(opts), _stream(),
                          ctypes.byref(h))
    if rc != ZOLO_OK and (rc not in allow or not h):
        raise ZoloError(rc, lib().zolo_last_error().decode())
    try:
        L = lib()
        cnt = L.zolo_result_count(h)
        ev = L.zolo_result_eigenvalues(h)
        eig = [ev[i] for i in range(cnt)]
        vec = torch.empty((pencil.n, max(cnt, 1)), dtype=torch.complex128 if pencil.cplx else torch.float64,
                          device=f"cuda:{ctx.device}")
        if cnt:
            _check(L.zolo_result_copy_vectors(h, _ptr(vec), vec.stride(0), _stream()))
        st = zolo_stats()
        _check(L.zolo_result_stats(h, ctypes.byref(st)))
    finally:
        lib().zolo_result_free(h)
    return eig, vec[:, :cnt], struct_dict(st), rc


def zolo_solve(ctx: Context, pencil: Pencil, a, b, n_lambda_est, opts: zolo_opts = None, Q0=None,
               allow=(ZOLO_ENOCONV,), host_vectors=False):
    """Returns (eigenvalues list, vectors N x count, stats dict, status).  The vectors
    are a device tensor (zolo_result_copy_vectors), or with host_vectors=True a numpy
    array (zolo_result_copy_vectors_host)."""
    import numpy as np
    import torch

    if opts is None:
        opts = zolo_opts_default()
    h = _vp()
    rc = lib().zolo_solve(ctx.h, pencil.h, float(a), float(b), int(n_lambda_est), ctypes.byref(opts),
                          None if Q0 is None else _ptr(Q0), _stream(), ctypes.byref(h))
    if rc != ZOLO_OK and (rc not in allow or not h):
        raise ZoloError(rc, lib().zolo_last_error().decode())
    try:
        L = lib()
        cnt = L.zolo_result_count(h)
        ev = L.zolo_result_eigenvalues(h)
        eig = [ev[i] for i in range(cnt)]
        if host_vectors:
            vec = np.empty((pencil.n, max(cnt, 1)), dtype=np.complex128 if pencil.cplx else np.float64)
            if cnt:
                _check(L.zolo_result_copy_vectors_host(h, _np_ptr(vec), vec.shape[1]))
        else:
            vec = torch.empty((pencil.n, max(cnt, 1)), dtype=torch.complex128 if pencil.cplx else torch.float64,
                              device=f"cuda:{ctx.device}")
            if cnt:
                _check(L.zolo_result_copy_vectors(h, _ptr(vec), vec.stride(0), _stream()))
        st = zolo_stats()
        _check(L.zolo_result_stats(h, ctypes.byref(st)))
    finally:
        lib().zolo_result_free(h)
    return eig, vec[:, :cnt], struct_dict(st), rc


class Server:
    """zolo_server_create: worker threads with their own streams, admission by a
    device-memory budget (bytes; 0 = 80% of free memory), batching of queries
    that share a filter."""

    def __init__(self, ctx: Context, slots: int = 4, budget_bytes: int = 0):
        import weakref

        h = _vp()
        _check(lib().zolo_server_create(ctx.h, int(slots), int(budget_bytes), ctypes.byref(h)))
        self.h = h
        self.ctx = ctx
        self._queries = weakref.WeakSet()
        # pencils the server has run queries on: its resident factorizations and
        # subspaces refer to them, so they stay alive until dropped or closed
        self._pencils = {}

    def submit(self, pencil: Pencil, a, b, n_lambda_est, opts: zolo_opts = None, Q0=None) -> "Query":
        """Q0: optional host numpy array N x n_ss (row-major; float64, or complex128 for
        complex pencils)."""
        import numpy as np

        if opts is None:
            opts = zolo_opts_default()
        q0 = None if Q0 is None else np.ascontiguousarray(Q0, dtype=np.complex128 if pencil.cplx else np.float64)
        h = _vp()
        _check(lib().zolo_submit(self.h, pencil.h, float(a), float(b), int(n_lambda_est), ctypes.byref(opts),
                                 None if q0 is None else _np_ptr(q0), ctypes.byref(h)))
        q = Query(h, pencil, self)
        self._queries.add(q)
        self._pencils[id(pencil)] = pencil
        return q

    def drop_pencil(self, pencil: Pencil):
        """zolo_server_drop_pencil: waits for the pencil's queued and running
        queries and frees its resident factorizations and subspaces."""
        _check(lib().zolo_server_drop_pencil(self.h, pencil.h))
        self._pencils.pop(id(pencil), None)

    def info(self) -> dict:
        inf = zolo_server_info()
        _check(lib().zolo_server_get_info(self.h, ctypes.byref(inf)))
        return struct_dict(inf)

    def close(self):
        """Frees the queries still held (waiting for them), then the server."""
        if getattr(self, "h", None) and _lib is not None:
            for q in list(self._queries):
                q.free()
            _lib.zolo_server_destroy(self.h)
            self.h = None
            self._pencils = {}

    def __del__(self):
        self.close()


class Query:
    def __init__(self, h, pencil: Pencil, server: Server):
        self.h, self.pencil, self.server = h, pencil, server

    def wait(self, timeout_ms: int = -1, allow=(ZOLO_ENOCONV,)):
        """Returns (eigenvalues, vectors N x count on the device, stats, status, info)."""
        import torch

        r = _vp()
        rc = lib().zolo_wait(self.h, int(timeout_ms), ctypes.byref(r))
        if rc == ZOLO_ETIMEOUT:
            raise ZoloError(rc, lib().zolo_last_error().decode())
        if rc != ZOLO_OK and (rc not in allow or not r):
            if r:
                lib().zolo_result_free(r)
            raise ZoloError(rc, lib().zolo_last_error().decode())
        try:
            L = lib()
            cnt = L.zolo_result_count(r)
            ev = L.zolo_result_eigenvalues(r)
            eig = [ev[i] for i in range(cnt)]
            vec = torch.empty((self.pencil.n, max(cnt, 1)), dtype=torch.complex128 if self.pencil.cplx else torch.float64,
                              device=f"cuda:{self.server.ctx.device}")
            if cnt:
                _check(L.zolo_result_copy_vectors(r, _ptr(vec), vec.stride(0), _stream()))
            st = zolo_stats()
            _check(L.zolo_result_stats(r, ctypes.byref(st)))
        finally:
            lib().zolo_result_free(r)
        return eig, vec[:, :cnt], struct_dict(st), rc, self.info()

    def info(self) -> dict:
        inf = zolo_query_info()
        _check(lib().zolo_query_get_info(self.h, ctypes.byref(inf)))
        return struct_dict(inf)

    def free(self):
        # a closed server has freed its queries already
        if getattr(self, "h", None) and _lib is not None and getattr(self.server, "h", None):
            _lib.zolo_query_free(self.h)
        self.h = None

    def __del__(self):
        self.free()


def zolo_profile_enable(on: bool = True):
    _check(lib().zolo_profile_enable(1 if on else 0))


def zolo_profile_query() -> dict:
    out = {}
    for i, name in enumerate(PROF_CLASSES):
        p = zolo_kernel_profile()
        _check(lib().zolo_profile_query(i, ctypes.byref(p)))
        out[name] = struct_dict(p)
    return out


def opts_from_window(w: dict, r1=2, r2=0, n_ss=0, precision=ZOLO_PREC_FP64, **kw) -> zolo_opts:
    o = zolo_opts_default()
    o.a_minus = w["a_minus"] if math.isfinite(w["a_minus"]) else -math.inf
    o.a_plus = w["a_plus"]
    o.b_minus = w["b_minus"]
    o.b_plus = w["b_plus"] if math.isfinite(w["b_plus"]) else math.inf
    o.r1 = r1
    o.r2 = r2
    o.n_ss = n_ss
    o.precision = precision
    for k, v in kw.items():
        setattr(o, k, v)
    return o
