"""ctypes declarations of include/tracemin.h (argument marshalling only).

The shared library is built in-tree by ``paper_1108_4509_amd/build.py``.  If
it is missing, importing this module raises: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtracemin.so")

# status codes
TM_OK, TM_EINVAL, TM_ENOMEM, TM_ENOTSPD, TM_ENOCONV, TM_ENAN, TM_EDEVICE, TM_ENOTSUP, TM_EAGAIN = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
TM_F64, TM_F32 = 0, 1
TM_FULL_DP, TM_FULL_SP, TM_MP2, TM_MIXED, TM_MIXED_BF16, TM_FULL_BF16, TM_MP1, TM_MP2_MP1 = range(8)
TM_CHECK_SYMMETRY, TM_DEVICE_PTRS = 1, 2

c_void_p = ctypes.c_void_p
c_int32 = ctypes.c_int32
c_int64 = ctypes.c_int64
c_double = ctypes.c_double

ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)


class tm_allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", c_void_p)]


class tm_stencil(ctypes.Structure):
    _fields_ = [("ndim", c_int32), ("dims", c_int32 * 3), ("order", c_int32),
                ("periodic", c_int32), ("kinetic_scale", c_double),
                ("V", ctypes.POINTER(c_double))]


PROGRESS_FN = ctypes.CFUNCTYPE(None, c_int32, c_double, c_double, c_int32, c_void_p)


class tm_opts(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("max_iter", c_int32), ("k_rot", c_int32),
                ("k_check", c_int32), ("precondition", c_int32), ("history", c_int32),
                ("transport", c_int32), ("graphs", c_int32),
                ("switch_tol", c_double), ("rise_tol", c_double), ("stall_tol", c_double),
                ("seed", ctypes.c_uint64), ("cheb_degree", c_int32), ("reserved", c_int32),
                ("cheb_shift", c_double), ("progress", PROGRESS_FN), ("progress_user", c_void_p)]


class tm_result(ctypes.Structure):
    _fields_ = [("E_G", c_double), ("rho", c_double), ("max_residual", c_double),
                ("frob_residual", c_double), ("orth_err", c_double), ("seconds", c_double),
                ("seconds_phase", c_double * 3),
                ("iterations", c_int32), ("iters_sp", c_int32), ("converged", c_int32),
                ("restarts", c_int32), ("rotations", c_int32), ("iters_phase2", c_int32)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["seconds_phase"] = list(self.seconds_phase)
        return d


class tm_server_opts(ctypes.Structure):
    _fields_ = [("device", c_int32), ("max_slots", c_int32), ("hbm_budget", ctypes.c_uint64),
                ("max_batch", c_int32), ("max_batch_cols", c_int32)]


class tm_request(ctypes.Structure):
    _fields_ = [("n", c_int64), ("rowptr", c_void_p), ("col", c_void_p), ("val", c_void_p),
                ("m", c_int32), ("reserved", c_int32), ("tol", c_double), ("C0", c_void_p),
                ("opts", ctypes.POINTER(tm_opts))]


class tm_server_stats(ctypes.Structure):
    _fields_ = [("submitted", c_int64), ("completed", c_int64), ("failed", c_int64),
                ("rejected", c_int64), ("queued", c_int64), ("running", c_int64),
                ("p50_latency_s", c_double), ("p99_latency_s", c_double),
                ("max_latency_s", c_double), ("mean_latency_s", c_double),
                ("span_s", c_double), ("solves_per_s", c_double),
                ("hbm_budget", ctypes.c_uint64), ("hbm_peak", ctypes.c_uint64),
                ("p50_wait_s", c_double), ("p99_wait_s", c_double),
                ("p50_service_s", c_double), ("p99_service_s", c_double),
                ("solver_runs", c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# name -> (restype, argtypes); mirrors include/tracemin.h
SIGNATURES = {
    "tm_leading_dim": (c_int32, [c_int32]),
    "tm_create": (c_int32, [c_int32, ctypes.POINTER(tm_allocator), c_void_p, ctypes.POINTER(c_void_p)]),
    "tm_destroy": (None, [c_void_p]),
    "tm_status_string": (ctypes.c_char_p, [c_int32]),
    "tm_last_error": (ctypes.c_char_p, []),
    "tm_set_matrix_csr": (c_int32, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p,
                                    ctypes.c_uint32, ctypes.POINTER(c_void_p)]),
    "tm_random_block": (c_int32, [c_void_p, c_int64, c_int32, ctypes.c_uint64, c_void_p]),
    "tm_set_matrix_stencil": (c_int32, [c_void_p, ctypes.POINTER(tm_stencil),
                                        ctypes.POINTER(c_void_p)]),
    "tm_free_matrix": (None, [c_void_p]),
    "tm_matrix_rows": (c_int64, [c_void_p]),
    "tm_opts_default": (None, [ctypes.POINTER(tm_opts)]),
    "tm_solve": (c_int32, [c_void_p, c_void_p, c_int32, c_double, ctypes.POINTER(tm_opts),
                           c_void_p, c_void_p, c_void_p, ctypes.POINTER(tm_result),
                           c_void_p, c_int32]),
    "tm_solve_generalized": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_double,
                                       ctypes.POINTER(tm_opts), c_void_p, c_void_p, c_void_p,
                                       ctypes.POINTER(tm_result), c_void_p, c_int32]),
    "tm_set_matrix_batch": (c_int32, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_int32,
                                      c_void_p, ctypes.c_uint32, ctypes.POINTER(c_void_p)]),
    "tm_batch_layout": (c_int32, [c_int32, c_int32, ctypes.POINTER(c_int32), ctypes.POINTER(c_int32)]),
    "tm_solve_batch": (c_int32, [c_void_p, c_void_p, c_int32, c_double, ctypes.POINTER(tm_opts),
                                 c_void_p, c_void_p, c_void_p, ctypes.POINTER(tm_result)]),
    "tm_spmm": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p]),
    "tm_gram": (c_int32, [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                          c_void_p]),
    "tm_gram_noalloc": (c_int32, [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                  c_void_p]),
    "tm_rotate": (c_int32, [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "tm_energy_grad": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_void_p,
                                 c_void_p, c_void_p, c_void_p, c_void_p]),
    "tm_orthonormalize": (c_int32, [c_void_p, c_int64, c_int32, c_int32, c_void_p]),
    "tm_cholesky_inverse": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "tm_sym_eig": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "tm_time_kernel": (c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32,
                                 ctypes.POINTER(c_double)]),
    "tm_solve_footprint": (c_int32, [c_int64, c_int64, c_int32, ctypes.POINTER(tm_opts),
                                     ctypes.POINTER(ctypes.c_uint64)]),
    "tm_server_create": (c_int32, [ctypes.POINTER(tm_server_opts), ctypes.POINTER(c_void_p)]),
    "tm_server_submit": (c_int32, [c_void_p, ctypes.POINTER(tm_request),
                                   ctypes.POINTER(ctypes.c_uint64)]),
    "tm_server_poll": (c_int32, [c_void_p, ctypes.c_uint64, ctypes.POINTER(tm_result), c_void_p]),
    "tm_server_wait": (c_int32, [c_void_p, ctypes.c_uint64, c_double, ctypes.POINTER(tm_result),
                                 c_void_p]),
    "tm_server_get_stats": (c_int32, [c_void_p, ctypes.POINTER(tm_server_stats)]),
    "tm_server_destroy": (None, [c_void_p]),
}

(TM_K_SPMM, TM_K_GRAM_SHIFT, TM_K_GRAM_SYM, TM_K_ROT_GRAD, TM_K_TRMM, TM_K_GRAM_MP2,
 TM_K_ROT_GRAD_MP2, TM_K_TRMM_MP2, TM_K_CHOL, TM_K_GRAM_BF16X3) = range(10)

_lib = None


def lib():
    """The loaded libtracemin.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with paper_1108_4509_amd/build.py "
                "(there is no non-HIP fallback)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


class TraceminError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        detail = L.tm_last_error().decode()
        msg = L.tm_status_string(status).decode()
        super().__init__(f"{where}: {msg} ({status}) {detail}")
        self.status = status


def check(status: int, where: str, allow=(TM_OK,)):
    if status not in allow:
        raise TraceminError(status, where)
    return status
