"""MI355X-native trace-minimization eigensolver (Tsuchida & Choe, arXiv 1108.4509).

Thin Python binding over the C ABI in include/tracemin.h.  PyTorch provides
device memory (the library's allocator hook is bound to torch's caching
allocator) and the stream; every step of the solver runs in the HIP kernels of
libtracemin.so.  Functions keep the C names without the ``tm_`` prefix.
"""

from __future__ import annotations

import atexit
import ctypes
import sys
import weakref
from typing import Optional

import numpy as np

from . import _abi
from ._abi import (TM_F32, TM_F64, TM_FULL_DP, TM_FULL_SP, TM_MIXED, TM_MP2,  # noqa: F401
                   TM_MIXED_BF16, TM_FULL_BF16, TM_MP1, TM_MP2_MP1, TM_CHECK_SYMMETRY,
                   TM_DEVICE_PTRS, TM_ENOCONV, TM_ENOTSPD, TM_EINVAL, TM_ENOTSUP, TM_OK,
                   TraceminError)

PRECISIONS = {"full_dp": TM_FULL_DP, "full_sp": TM_FULL_SP, "mp2": TM_MP2, "mixed": TM_MIXED,
              "mixed_bf16": TM_MIXED_BF16, "full_bf16": TM_FULL_BF16, "mp1": TM_MP1,
              "mp2_mp1": TM_MP2_MP1}


def _torch():
    import torch
    return torch


# Matrices must be freed before their context is destroyed.  At interpreter
# exit the garbage collector gives no such order, so live handles are
# released explicitly by an exit hook registered after torch is imported (the
# hooks run in reverse order, so ours runs while torch is still usable).
_live_matrices: "weakref.WeakSet" = weakref.WeakSet()
_live_contexts: "weakref.WeakSet" = weakref.WeakSet()
_exit_hook_installed = False


def _release_all():
    for mat in list(_live_matrices):
        mat.free()
    for ctx in list(_live_contexts):
        ctx.close()


def leading_dim(m: int) -> int:
    return int(_abi.lib().tm_leading_dim(int(m)))


def _ptr(t) -> int:
    return int(t.data_ptr()) if t is not None else 0


class Context:
    """A library context on one GPU, using torch's allocator and current stream."""

    def __init__(self, device: int = 0, torch_allocator: bool = True):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the trace-minimization library needs a HIP device")
        self.device = int(device)
        torch.cuda.set_device(self.device)
        self.stream = torch.cuda.current_stream(self.device)
        L = _abi.lib()
        self._alloc = None
        alloc_ptr = None
        if torch_allocator:
            dev, stream = self.device, self.stream

            def _a(nbytes, _user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
                except Exception:  # reported to the library as a failed allocation
                    return None

            def _f(ptr, _user):
                torch.cuda.caching_allocator_delete(int(ptr))

            self._alloc = _abi.tm_allocator(_abi.ALLOC_FN(_a), _abi.FREE_FN(_f), None)
            alloc_ptr = ctypes.byref(self._alloc)
        h = ctypes.c_void_p()
        _abi.check(L.tm_create(self.device, alloc_ptr, ctypes.c_void_p(self.stream.cuda_stream),
                               ctypes.byref(h)), "tm_create")
        self.handle = h
        global _exit_hook_installed
        if not _exit_hook_installed:
            atexit.register(_release_all)
            _exit_hook_installed = True
        _live_contexts.add(self)

    def close(self):
        if getattr(self, "handle", None):
            for mat in list(_live_matrices):
                if mat.ctx is self:
                    mat.free()
            _abi.lib().tm_destroy(self.handle)
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # the default argument keeps the check usable while module globals
        # are being torn down at interpreter exit
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


class Matrix:
    """A device-resident H (CSR or stencil) owned by a Context."""

    def __init__(self, ctx: Context, handle: ctypes.c_void_p, n: int):
        self.ctx, self.handle, self.n = ctx, handle, n
        self.batch_k = 0
        _live_matrices.add(self)

    def free(self):
        if self.handle and self.ctx.handle:
            _abi.lib().tm_free_matrix(self.handle)
        self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


def set_matrix_csr(ctx: Context, rowptr, col, val, check_symmetry: bool = False) -> Matrix:
    """H from CSR arrays: numpy host arrays, or torch device tensors (then
    passed as device pointers, TM_DEVICE_PTRS)."""
    torch = _torch()
    flags = TM_CHECK_SYMMETRY if check_symmetry else 0
    if isinstance(rowptr, torch.Tensor):
        if (rowptr.dtype, col.dtype, val.dtype) != (torch.int64, torch.int32, torch.float64):
            raise ValueError("device CSR arrays must be int64, int32 and float64")
        if not (rowptr.is_cuda and col.is_cuda and val.is_cuda):
            raise ValueError("tensor CSR arrays must live on the device")
        rowptr, col, val = rowptr.contiguous(), col.contiguous(), val.contiguous()
        n = rowptr.shape[0] - 1
        ptrs = (rowptr.data_ptr(), col.data_ptr(), val.data_ptr())
        flags |= TM_DEVICE_PTRS
    else:
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        n = rowptr.shape[0] - 1
        ptrs = (rowptr.ctypes.data, col.ctypes.data, val.ctypes.data)
    h = ctypes.c_void_p()
    _abi.check(_abi.lib().tm_set_matrix_csr(ctx.handle, n, *ptrs, flags, ctypes.byref(h)),
               "tm_set_matrix_csr")
    return Matrix(ctx, h, n)


def set_matrix_stencil(ctx: Context, ndim: int, dims, order: int = 2, periodic: bool = True,
                       kinetic_scale: float = 0.5, V: Optional[np.ndarray] = None) -> Matrix:
    s = _abi.tm_stencil()
    s.ndim = ndim
    d = list(dims) + [1] * (3 - len(dims))
    for i in range(3):
        s.dims[i] = int(d[i])
    s.order = order
    s.periodic = 1 if periodic else 0
    s.kinetic_scale = kinetic_scale
    keep = None
    if V is not None:
        keep = np.ascontiguousarray(V, dtype=np.float64).reshape(-1)
        s.V = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    h = ctypes.c_void_p()
    _abi.check(_abi.lib().tm_set_matrix_stencil(ctx.handle, ctypes.byref(s), ctypes.byref(h)),
               "tm_set_matrix_stencil")
    n = int(np.prod(d[:ndim]))
    return Matrix(ctx, h, n)


def matrix_from_problem(ctx: Context, problem, stencil: bool = False) -> Matrix:
    """Upload a ``workloads.Problem`` as CSR or as a stencil."""
    if stencil:
        sp = problem.spec
        return set_matrix_stencil(ctx, sp.ndim, sp.dims, sp.order, sp.bc == "periodic",
                                  sp.kinetic_scale, problem.V)
    return set_matrix_csr(ctx, *problem.csr())


def to_block(C: np.ndarray, dtype=None, device=None):
    """N x m host array -> zero-padded N x ld device tensor (FP64 unless dtype)."""
    torch = _torch()
    N, m = C.shape
    ld = leading_dim(m)
    dt = dtype or torch.float64
    out = torch.zeros((N, ld), dtype=dt, device=device or "cuda")
    out[:, :m] = torch.from_numpy(np.ascontiguousarray(C)).to(out.device, dt)
    return out


def random_block(ctx: Context, n: int, m: int, seed: int):
    """The seeded standard normal N x ld start block (tm_random_block)."""
    torch = _torch()
    out = torch.empty((n, leading_dim(m)), dtype=torch.float64, device="cuda")
    _abi.check(_abi.lib().tm_random_block(ctx.handle, n, m, int(seed), _ptr(out)), "tm_random_block")
    return out


def opts(precision="full_dp", max_iter=20000, k_rot=50, k_check=10, precondition=False,
         history=False, switch_tol=0.0, rise_tol=1e-13, transport=None,
         stall_tol=0.0, graphs=None, seed=0, cheb_degree=None, cheb_shift=None,
         progress=None) -> _abi.tm_opts:
    """tm_opts; precondition: False, True / "diagonal" (Eq. 18 with the
    diagonal M) or "chebyshev" (the polynomial M of cheb_degree steps).
    progress: optional callable(iterations, E, rho, phase), called at each
    host poll of a running solve."""
    o = _abi.tm_opts()
    _abi.lib().tm_opts_default(ctypes.byref(o))
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.max_iter = max_iter
    o.k_rot = k_rot
    o.k_check = k_check
    o.precondition = 2 if precondition == "chebyshev" else (1 if precondition else 0)
    if cheb_degree is not None:
        o.cheb_degree = int(cheb_degree)
    if cheb_shift is not None:
        o.cheb_shift = float(cheb_shift)
    o.history = 1 if history else 0
    o.switch_tol = switch_tol
    o.rise_tol = rise_tol
    o.stall_tol = stall_tol
    if graphs is not None:
        o.graphs = 1 if graphs else 0
    if transport is not None:
        o.transport = 1 if transport else 0
    o.seed = int(seed)
    if progress is not None:
        cb = _abi.PROGRESS_FN(lambda it, E, rho, ph, _u: progress(it, E, rho, ph))
        o.progress = cb
        o._keep_progress = cb     # the C function pointer lives as long as the options
    return o


def solve(ctx: Context, H: Matrix, m: int, tol: float, C0, options=None, history_len: int = 0,
          want_vectors: bool = True, allow_noconv: bool = True, S: Optional[Matrix] = None):
    """Run tm_solve.  C0: N x ld FP64 device tensor (see ``to_block``), or
    None for the seeded start block of ``options.seed``.

    Returns (result dict, C tensor or None, eigenvalue tensor, history array or None).
    """
    torch = _torch()
    if C0 is not None:
        N, ld = C0.shape
        if C0.dtype != torch.float64 or not C0.is_contiguous():
            raise ValueError("C0 must be a contiguous FP64 device tensor")
    else:
        N, ld = H.n, leading_dim(m)
    o = options or opts()
    Cout = (torch.empty((N, ld), dtype=torch.float64, device="cuda") if want_vectors else None)
    eig = torch.empty(max(m, 1), dtype=torch.float64, device="cuda")
    hist = np.zeros(2 * history_len) if history_len > 0 else None
    res = _abi.tm_result()
    hp = hist.ctypes.data if hist is not None else None
    if S is None:
        st = _abi.lib().tm_solve(ctx.handle, H.handle, m, tol, ctypes.byref(o), _ptr(C0), _ptr(Cout),
                                 _ptr(eig), ctypes.byref(res), hp, history_len)
    else:
        # H x = lambda S x (tm_solve_generalized)
        st = _abi.lib().tm_solve_generalized(ctx.handle, H.handle, S.handle, m, tol, ctypes.byref(o),
                                             _ptr(C0), _ptr(Cout), _ptr(eig), ctypes.byref(res), hp,
                                             history_len)
    _abi.check(st, "tm_solve", allow=(TM_OK, TM_ENOCONV) if allow_noconv else (TM_OK,))
    r = res.as_dict()
    r["status"] = st
    if hist is not None:
        n = min(history_len, r["iterations"] + (1 if r["converged"] else 0))
        hist = hist.reshape(-1, 2)[:n]
    return r, Cout, eig[:m], hist


# ------------------------------------------------------------- batches

def batch_layout(k: int, m: int):
    """(ldg, ld): problem g of a batch of k owns columns g*ldg .. g*ldg+m-1
    of an N x ld block (tm_batch_layout)."""
    ldg, ld = ctypes.c_int32(), ctypes.c_int32()
    _abi.check(_abi.lib().tm_batch_layout(k, m, ctypes.byref(ldg), ctypes.byref(ld)), "tm_batch_layout")
    return ldg.value, ld.value


def set_matrix_batch(ctx: Context, rowptr, col, val, d, check_symmetry: bool = False) -> Matrix:
    """k operators H_g = A + diag(d[g]) sharing the CSR A (host arrays); d is
    a k x N host array (tm_set_matrix_batch)."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    d = np.ascontiguousarray(np.atleast_2d(d), dtype=np.float64)
    n = rowptr.shape[0] - 1
    if d.shape[1] != n:
        raise ValueError("d must be k x N")
    h = ctypes.c_void_p()
    flags = TM_CHECK_SYMMETRY if check_symmetry else 0
    _abi.check(_abi.lib().tm_set_matrix_batch(ctx.handle, n, rowptr.ctypes.data, col.ctypes.data,
                                              val.ctypes.data, d.shape[0], d.ctypes.data, flags,
                                              ctypes.byref(h)), "tm_set_matrix_batch")
    M = Matrix(ctx, h, n)
    M.batch_k = d.shape[0]
    return M


def solve_batch(ctx: Context, H: Matrix, m: int, tol: float, C0=None, options=None,
                want_vectors: bool = True, allow_noconv: bool = True):
    """Run tm_solve_batch on a batch matrix.  C0: N x ld FP64 device tensor in
    the batch layout, or None (problem g from seed options.seed + g).

    Returns (list of k result dicts, C tensor or None, k x m eigenvalue tensor)."""
    torch = _torch()
    k = H.batch_k
    _, ld = batch_layout(k, m)
    if C0 is not None and (C0.dtype != torch.float64 or not C0.is_contiguous() or C0.shape != (H.n, ld)):
        raise ValueError("C0 must be a contiguous N x ld FP64 device tensor")
    o = options or opts()
    Cout = torch.empty((H.n, ld), dtype=torch.float64, device="cuda") if want_vectors else None
    eig = torch.empty((k, m), dtype=torch.float64, device="cuda")
    res = (_abi.tm_result * k)()
    st = _abi.lib().tm_solve_batch(ctx.handle, H.handle, m, tol, ctypes.byref(o), _ptr(C0), _ptr(Cout),
                                   _ptr(eig), res)
    _abi.check(st, "tm_solve_batch", allow=(TM_OK, TM_ENOCONV) if allow_noconv else (TM_OK,))
    out = []
    for r in res:
        d = r.as_dict()
        d["status"] = st
        out.append(d)
    return out, Cout, eig


# ------------------------------------------------------------- single steps

def _dtype_code(t):
    torch = _torch()
    return TM_F64 if t.dtype == torch.float64 else TM_F32


def spmm(ctx: Context, H: Matrix, m: int, C, X):
    _abi.check(_abi.lib().tm_spmm(ctx.handle, H.handle, m, _dtype_code(C), _ptr(C), _ptr(X)),
               "tm_spmm")


def gram(ctx: Context, m: int, A, B, h=None, out=None, bf16x3: bool = False):
    """A^T (B - A diag(h)) (h optional), m x m FP64.  bf16x3: FP32 blocks on
    BF16 matrix cores with two-term BF16 operands."""
    torch = _torch()
    n = A.shape[0]
    out = out if out is not None else torch.empty((m, m), dtype=torch.float64, device=A.device)
    code = _dtype_code(A)
    if bf16x3:
        if A.dtype != torch.float32:
            raise ValueError("bf16x3 takes FP32 blocks")
        code = 2
    _abi.check(_abi.lib().tm_gram(ctx.handle, n, m, code, _ptr(A), _ptr(B), _ptr(h),
                                  _ptr(out)), "tm_gram")
    return out


def gram_noalloc(ctx: Context, m: int, A, B, h=None, out=None, bf16x3: bool = False):
    """tm_gram_noalloc: as ``gram`` with no device allocation inside the
    library (enqueue only; synchronize the stream before reading out)."""
    torch = _torch()
    n = A.shape[0]
    out = out if out is not None else torch.empty((m, m), dtype=torch.float64, device=A.device)
    code = _dtype_code(A)
    if bf16x3:
        if A.dtype != torch.float32:
            raise ValueError("bf16x3 takes FP32 blocks")
        code = 2
    _abi.check(_abi.lib().tm_gram_noalloc(ctx.handle, n, m, code, _ptr(A), _ptr(B), _ptr(h),
                                          _ptr(out)), "tm_gram_noalloc")
    return out


def rotate(ctx: Context, m: int, A, W, out=None):
    torch = _torch()
    out = out if out is not None else torch.empty_like(A)
    _abi.check(_abi.lib().tm_rotate(ctx.handle, A.shape[0], m, _dtype_code(A), _ptr(A), _ptr(W),
                                    _ptr(out)), "tm_rotate")
    return out


def energy_grad(ctx: Context, H: Matrix, m: int, C, precision="full_dp"):
    torch = _torch()
    X = torch.empty_like(C)
    G = torch.empty_like(C)
    h = torch.empty(m, dtype=torch.float64, device=C.device)
    Hp = torch.empty((m, m), dtype=torch.float64, device=C.device)
    E = torch.empty(1, dtype=torch.float64, device=C.device)
    p = PRECISIONS[precision] if isinstance(precision, str) else precision
    _abi.check(_abi.lib().tm_energy_grad(ctx.handle, H.handle, m, p, _ptr(C), _ptr(X), _ptr(G),
                                         _ptr(h), _ptr(Hp), _ptr(E)), "tm_energy_grad")
    return float(E.item()), G, X, h, Hp


def orthonormalize(ctx: Context, m: int, C, precision="full_dp"):
    p = PRECISIONS[precision] if isinstance(precision, str) else precision
    _abi.check(_abi.lib().tm_orthonormalize(ctx.handle, C.shape[0], m, p, _ptr(C)),
               "tm_orthonormalize")
    return C


def cholesky_inverse(ctx: Context, S):
    torch = _torch()
    m = S.shape[0]
    R = torch.empty_like(S)
    _abi.check(_abi.lib().tm_cholesky_inverse(ctx.handle, m, _ptr(S), _ptr(R)),
               "tm_cholesky_inverse")
    return R


def sym_eig(ctx: Context, A):
    torch = _torch()
    m = A.shape[0]
    U = torch.empty_like(A)
    w = torch.empty(m, dtype=torch.float64, device=A.device)
    _abi.check(_abi.lib().tm_sym_eig(ctx.handle, m, _ptr(A), _ptr(U), _ptr(w)), "tm_sym_eig")
    return w, U


KERNELS = {"spmm": _abi.TM_K_SPMM, "gram_shift": _abi.TM_K_GRAM_SHIFT,
           "gram_sym": _abi.TM_K_GRAM_SYM, "rot_grad": _abi.TM_K_ROT_GRAD,
           "trmm": _abi.TM_K_TRMM, "gram_mp2": _abi.TM_K_GRAM_MP2,
           "rot_grad_mp2": _abi.TM_K_ROT_GRAD_MP2, "trmm_mp2": _abi.TM_K_TRMM_MP2,
           "chol": _abi.TM_K_CHOL, "gram_bf16x3": _abi.TM_K_GRAM_BF16X3}


def time_kernel(ctx: Context, H: Matrix, kernel: str, m: int, dtype: str = "f32",
                reps: int = 20) -> float:
    """Average duration (ms) of one kernel launch, timed with HIP events."""
    out = ctypes.c_double()
    code = TM_F64 if dtype == "f64" else TM_F32
    _abi.check(_abi.lib().tm_time_kernel(ctx.handle, H.handle, KERNELS[kernel], m, code, reps,
                                         ctypes.byref(out)), "tm_time_kernel")
    return out.value


# ------------------------------------------------------------------ serving

def solve_footprint(n: int, nnz: int, m: int, options=None) -> int:
    """Device bytes the server reserves for one request (tm_solve_footprint)."""
    out = ctypes.c_uint64()
    o = ctypes.byref(options) if options is not None else None
    _abi.check(_abi.lib().tm_solve_footprint(n, nnz, m, o, ctypes.byref(out)), "tm_solve_footprint")
    return out.value


class Server:
    """Continuous-batching solve server (tm_server_*): requests are host CSR
    matrices with a host start block; results are host eigenvalues."""

    def __init__(self, device: int = 0, max_slots: int = 4, hbm_budget: int = 16 << 30,
                 max_batch: int = 0, max_batch_cols: int = 0):
        o = _abi.tm_server_opts(device=device, max_slots=max_slots, hbm_budget=hbm_budget,
                                max_batch=max_batch, max_batch_cols=max_batch_cols)
        h = ctypes.c_void_p()
        _abi.check(_abi.lib().tm_server_create(ctypes.byref(o), ctypes.byref(h)), "tm_server_create")
        self.handle = h
        self._keep = {}

    def submit(self, rowptr, col, val, m: int, tol: float, C0, options=None) -> int:
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        C0 = np.ascontiguousarray(C0, dtype=np.float64)
        n = len(rowptr) - 1
        if C0.shape != (n, m):
            raise ValueError("C0 must be n x m")
        req = _abi.tm_request(n=n, rowptr=rowptr.ctypes.data, col=col.ctypes.data,
                              val=val.ctypes.data, m=m, reserved=0, tol=tol,
                              C0=C0.ctypes.data,
                              opts=ctypes.pointer(options) if options is not None else None)
        rid = ctypes.c_uint64()
        _abi.check(_abi.lib().tm_server_submit(self.handle, ctypes.byref(req), ctypes.byref(rid)),
                   "tm_server_submit")
        self._keep[rid.value] = m
        return rid.value

    def _result(self, fn, rid: int, *args):
        m = self._keep[rid]
        res = _abi.tm_result()
        eig = np.zeros(m)
        st = fn(self.handle, rid, *args, ctypes.byref(res), eig.ctypes.data)
        if st == _abi.TM_EAGAIN:
            return None
        del self._keep[rid]
        _abi.check(st, "served solve", allow=(_abi.TM_OK, _abi.TM_ENOCONV))
        d = res.as_dict()
        d["status"] = st
        return d, eig

    def poll(self, rid: int):
        """(result dict, eigenvalues) once finished, else None."""
        return self._result(_abi.lib().tm_server_poll, rid)

    def wait(self, rid: int, timeout: float = -1.0):
        return self._result(_abi.lib().tm_server_wait, rid, float(timeout))

    def stats(self) -> dict:
        s = _abi.tm_server_stats()
        _abi.check(_abi.lib().tm_server_get_stats(self.handle, ctypes.byref(s)), "tm_server_get_stats")
        return s.as_dict()

    def close(self):
        if getattr(self, "handle", None):
            _abi.lib().tm_server_destroy(self.handle)
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass
