"""Python binding of libfdgmres.so: argument marshalling only.

Every computation runs in the library (host setup in C++, the solve in HIP kernels);
torch tensors provide device memory and the HIP stream.  The names follow the C ABI in
include/fdgmres.h.  The library must have been built (``build.build()``); importing
this module without it raises, there is no fallback.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdgmres.so")

FDG_OK = 0
FDG_NOT_CONVERGED = 1
FDG_EFULL = -7
PREC_FP64, PREC_FP32, PREC_BF16 = 0, 1, 2
SOLVE_USE_X0 = 1
SOLVE_FIXED_ITERS = 2
SOLVE_NO_AHEAD = 4
SOLVE_TIME_SPLIT = 8
TIMER_APPLY, TIMER_MATVEC, TIMER_KRYLOV, TIMER_FIBRE, TIMER_RESIDUAL = 0, 1, 2, 3, 4

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)


class FdgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class fdg_info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("converged", ctypes.c_int),
                ("breakdown", ctypes.c_int), ("rel_res_est", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("ms_total", ctypes.c_double), ("half_steps", ctypes.c_int),
                ("t_apply_ms", ctypes.c_double), ("t_matvec_ms", ctypes.c_double), ("t_orth_ms", ctypes.c_double),
                ("t_host_ms", ctypes.c_double)]


class fdg_done(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("status", ctypes.c_int), ("info", fdg_info)]


_lib = None

EXPORTS = [
    "fdg_colloc_factors", "fdg_factor_pencil", "fdg_deformed_csr", "fdg_manufactured_rhs",
    "fdg_create", "fdg_destroy", "fdg_set_prec_factors", "fdg_set_precision",
    "fdg_set_operator_kron", "fdg_set_operator_csr", "fdg_apply_prec", "fdg_matvec", "fdg_solve",
    "fdg_footprint_bytes", "fdg_timer_enable", "fdg_timer_read", "fdg_status_str", "fdg_last_error",
    "fdg_server_create", "fdg_server_destroy", "fdg_server_run_bytes", "fdg_server_admit", "fdg_server_step",
    "fdg_server_pending", "fdg_server_stats", "fdg_set_operator_mapped", "fdg_set_operator_fields",
    "fdg_deformed_coefficients", "fdg_factor_pencil_sym", "fdg_galerkin_factors", "fdg_galerkin_csr",
    "fdg_set_prec_factors_sym", "fdg_bicgstab", "fdg_operator_bytes", "fdg_factor_pencil_blocks",
    "fdg_set_prec_factors_blocks", "fdg_apply_prec_noalloc", "fdg_ctx_bytes", "fdg_release_workspace",
    "fdg_workspace_bytes", "fdg_attach_workspace",
]


def lib():
    """Loads the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} not built: run paper_1705_04384_amd/build.py (no fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    L.fdg_colloc_factors.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp]
    L.fdg_factor_pencil.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp]
    L.fdg_deformed_csr.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int, _i64p, _i64p,
                                   _i32p, _dp]
    L.fdg_manufactured_rhs.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp]
    L.fdg_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, _i32p, ctypes.c_int, ctypes.c_void_p]
    L.fdg_destroy.argtypes = [ctypes.c_void_p]
    L.fdg_set_prec_factors.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]
    L.fdg_set_precision.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.fdg_set_operator_kron.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp]
    L.fdg_set_operator_csr.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _dp]
    L.fdg_apply_prec.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.fdg_apply_prec_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.fdg_matvec.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    L.fdg_solve.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                            ctypes.c_int, ctypes.c_int, ctypes.POINTER(fdg_info)]
    L.fdg_footprint_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.fdg_footprint_bytes.restype = ctypes.c_size_t
    L.fdg_timer_enable.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
    L.fdg_timer_read.argtypes = [ctypes.c_void_p, ctypes.c_int, _i64p, _dp]
    L.fdg_server_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_size_t]
    L.fdg_server_destroy.argtypes = [ctypes.c_void_p]
    L.fdg_server_run_bytes.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.fdg_server_run_bytes.restype = ctypes.c_size_t
    L.fdg_server_admit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int64]
    L.fdg_server_step.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(fdg_done), ctypes.c_int,
                                  ctypes.POINTER(ctypes.c_int)]
    L.fdg_server_pending.argtypes = [ctypes.c_void_p]
    L.fdg_server_stats.argtypes = [ctypes.c_void_p, _i64p, _i64p, _i64p, _i64p]
    L.fdg_set_operator_mapped.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp]
    L.fdg_set_operator_fields.argtypes = [ctypes.c_void_p, _dp]
    L.fdg_deformed_coefficients.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp]
    L.fdg_factor_pencil_blocks.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.fdg_set_prec_factors_blocks.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp, _dp, _dp]
    L.fdg_factor_pencil_sym.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp]
    L.fdg_galerkin_factors.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
    L.fdg_galerkin_csr.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, ctypes.c_double, _i64p,
                                   _i64p, _i32p, _dp]
    L.fdg_set_prec_factors_sym.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp]
    L.fdg_operator_bytes.argtypes = [ctypes.c_void_p]
    L.fdg_operator_bytes.restype = ctypes.c_size_t
    L.fdg_ctx_bytes.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    L.fdg_release_workspace.argtypes = [ctypes.c_void_p]
    L.fdg_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.fdg_workspace_bytes.restype = ctypes.c_size_t
    L.fdg_attach_workspace.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    L.fdg_bicgstab.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_int,
                               ctypes.c_int, ctypes.POINTER(fdg_info)]
    L.fdg_status_str.argtypes = [ctypes.c_int]
    L.fdg_status_str.restype = ctypes.c_char_p
    L.fdg_last_error.argtypes = []
    L.fdg_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(st, allow=(FDG_OK,)):
    if st in allow:
        return st
    L = lib()
    raise FdgError(st, f"{L.fdg_status_str(st).decode()}: {L.fdg_last_error().decode()}")


def _ptr(a, typ=_dp):
    return a.ctypes.data_as(typ)


# ---- host setup -------------------------------------------------------------------------

def colloc_factors(p, n):
    """(M, K, D1, tau) of eq. 2.8 on the uniform open knot vector, Greville points (eq. 2.4)."""
    M = np.zeros((n, n)); K = np.zeros((n, n)); D1 = np.zeros((n, n)); tau = np.zeros(n)
    _check(lib().fdg_colloc_factors(p, n, _ptr(M), _ptr(K), _ptr(D1), _ptr(tau)))
    return M, K, D1, tau


def factor_pencil(K, M, want_cond=True):
    """(U, V, lam, cond1(U)) with K U = M U diag(lam), V = (M U)^{-T} (eq. 4.6); the
    condition number (an extra factorisation) is None unless want_cond."""
    K = np.ascontiguousarray(K, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    n = K.shape[0]
    U = np.zeros((n, n)); V = np.zeros((n, n)); lam = np.zeros(n); c = ctypes.c_double()
    _check(lib().fdg_factor_pencil(n, _ptr(K), _ptr(M), _ptr(U), _ptr(V), _ptr(lam),
                                   ctypes.byref(c) if want_cond else None))
    return U, V, lam, (c.value if want_cond else None)


def factor_pencil_blocks(K, M, want_cond=False):
    """(U, V, lam, mu, cond1(U)): K U = M U D with D block diagonal (2x2 blocks
    [[lam_c, mu_c], [mu_{c+1}, lam_{c+1}]] for complex pairs), V = (M U)^{-T}."""
    K = np.ascontiguousarray(K, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    n = K.shape[0]
    U = np.zeros((n, n)); V = np.zeros((n, n)); lam = np.zeros(n); mu = np.zeros(n); c = ctypes.c_double()
    _check(lib().fdg_factor_pencil_blocks(n, _ptr(K), _ptr(M), _ptr(U), _ptr(V), _ptr(lam), _ptr(mu),
                                          ctypes.byref(c) if want_cond else None))
    return U, V, lam, mu, (c.value if want_cond else None)


def factor_pencil_sym(K, M):
    """(U, lam) with K U = M U diag(lam), U^T M U = I: the symmetric FD factors (V = U)."""
    K = np.ascontiguousarray(K, dtype=np.float64)
    M = np.ascontiguousarray(M, dtype=np.float64)
    n = K.shape[0]
    U = np.zeros((n, n)); lam = np.zeros(n)
    _check(lib().fdg_factor_pencil_sym(n, _ptr(K), _ptr(M), _ptr(U), _ptr(lam)))
    return U, lam


def galerkin_factors(p, n, w0=0.0, w1=0.0):
    """(M, K, H): univariate Galerkin factors of eq. 3.8 and the convection factor of the
    affine wind w0 + w1 z (after eq. 3.9)."""
    M = np.zeros((n, n)); K = np.zeros((n, n)); H = np.zeros((n, n))
    _check(lib().fdg_galerkin_factors(p, n, w0, w1, _ptr(M), _ptr(K), _ptr(H)))
    return M, K, H


def galerkin_csr(p, n, amp=0.0, wind=None, beta=0.0):
    """CSR (rowptr, col, val) of the Galerkin matrix of -Lap u + w . grad u on the
    deformed cube (wind = (c_1, c_2, c_3) or None)."""
    L = lib()
    w = None if wind is None else np.ascontiguousarray(wind, dtype=np.float64)
    wp = None if w is None else _ptr(w)
    nnz = ctypes.c_int64()
    _check(L.fdg_galerkin_csr(p, n, amp, wp, beta, ctypes.byref(nnz), None, None, None))
    rowptr = np.zeros(n ** 3 + 1, dtype=np.int64)
    col = np.zeros(nnz.value, dtype=np.int32)
    val = np.zeros(nnz.value, dtype=np.float64)
    _check(L.fdg_galerkin_csr(p, n, amp, wp, beta, ctypes.byref(nnz), _ptr(rowptr, _i64p), _ptr(col, _i32p),
                              _ptr(val)))
    return rowptr, col, val


def deformed_csr(p, n, amp=0.1, band=False):
    """CSR (rowptr, col, val) of the collocation matrix on the deformed cube."""
    L = lib()
    nnz = ctypes.c_int64()
    _check(L.fdg_deformed_csr(p, n, amp, int(band), ctypes.byref(nnz), None, None, None))
    rowptr = np.zeros(n ** 3 + 1, dtype=np.int64)
    col = np.zeros(nnz.value, dtype=np.int32)
    val = np.zeros(nnz.value, dtype=np.float64)
    _check(L.fdg_deformed_csr(p, n, amp, int(band), ctypes.byref(nnz), _ptr(rowptr, _i64p), _ptr(col, _i32p),
                              _ptr(val)))
    return rowptr, col, val


def deformed_coefficients(p, n, amp=0.1):
    """The 9 coefficient fields (9, n^3) of the deformed-cube operator at the collocation
    points: C_11, C_22, C_33, 2 C_12, 2 C_13, 2 C_23, g_1, g_2, g_3."""
    coef = np.zeros(9 * n ** 3)
    _check(lib().fdg_deformed_coefficients(p, n, amp, _ptr(coef)))
    return coef.reshape(9, n ** 3)


def manufactured_rhs(d, n, tau):
    f = np.zeros(n ** d)
    _check(lib().fdg_manufactured_rhs(d, n, _ptr(np.ascontiguousarray(tau, dtype=np.float64)), _ptr(f)))
    return f


def footprint_bytes(d, n, batch=1, prec=PREC_FP64, restart=30):
    return int(lib().fdg_footprint_bytes(d, n, batch, prec, restart))


# ---- device context -------------------------------------------------------------------------

_torch = None


def server_run_bytes(ctx, restart=30):
    """Arena bytes one request of this context takes in a server of the given restart."""
    return int(lib().fdg_server_run_bytes(ctx._h, restart))


def workspace_bytes(d, n, batch=1, restart=30):
    """Bytes of a buffer Context.attach_workspace accepts for this shape and restart."""
    return int(lib().fdg_workspace_bytes(d, n, batch, restart))


def _dev_ptr(t, numel, device):
    """Device address of t after checking that it is a contiguous float64 tensor of exactly
    numel elements on CUDA device index `device` (the C ABI takes bare pointers, so an
    undersized or foreign tensor would be read or written out of bounds)."""
    global _torch
    if _torch is None:
        import torch
        _torch = torch
    if not isinstance(t, _torch.Tensor):
        raise ValueError("expected a torch tensor")
    if t.dtype != _torch.float64 or not t.is_contiguous():
        raise ValueError("expected a contiguous float64 tensor")
    if t.numel() != numel:
        raise ValueError(f"expected {numel} elements, got {t.numel()}")
    if not t.is_cuda:
        raise ValueError("expected a CUDA tensor")
    if t.device.index != device:
        raise ValueError(f"tensor on cuda:{t.device.index}, context on cuda:{device}")
    return t.data_ptr()


class Context:
    """One problem shape (d, n, batch) on one HIP stream."""

    def __init__(self, d, n, batch=1, stream=None):
        import torch
        self.d, self.n, self.batch = d, n, batch
        self.N = n ** d
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.device = torch.cuda.current_device()
        h = ctypes.c_void_p()
        dims = (ctypes.c_int32 * 3)(n, n, n)
        _check(lib().fdg_create(ctypes.byref(h), d, dims, batch, ctypes.c_void_p(stream.cuda_stream)))
        self._h = h
        self._ws = None  # an attached workspace buffer, kept alive while attached

    def close(self):
        if self._h:
            lib().fdg_destroy(self._h)
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_prec_factors(self, l, U, V, lam):
        U = np.ascontiguousarray(U, dtype=np.float64)
        V = np.ascontiguousarray(V, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        _check(lib().fdg_set_prec_factors(self._h, l, _ptr(U), _ptr(V), _ptr(lam)))

    def set_prec_factors_blocks(self, l, U, V, lam, mu):
        U, V, lam, mu = (np.ascontiguousarray(a, dtype=np.float64) for a in (U, V, lam, mu))
        _check(lib().fdg_set_prec_factors_blocks(self._h, l, _ptr(U), _ptr(V), _ptr(lam), _ptr(mu)))

    def set_prec_factors_sym(self, l, U, lam):
        U = np.ascontiguousarray(U, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        _check(lib().fdg_set_prec_factors_sym(self._h, l, _ptr(U), _ptr(lam)))

    def set_precision(self, prec):
        _check(lib().fdg_set_precision(self._h, prec))

    def set_operator_kron(self, l, M, K):
        M = np.ascontiguousarray(M, dtype=np.float64)
        K = np.ascontiguousarray(K, dtype=np.float64)
        _check(lib().fdg_set_operator_kron(self._h, l, _ptr(M), _ptr(K)))

    def set_operator_csr(self, rowptr, col, val):
        rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        _check(lib().fdg_set_operator_csr(self._h, len(rowptr) - 1, len(col), _ptr(rowptr, _i64p),
                                          _ptr(col, _i32p), _ptr(val)))

    def set_operator_mapped(self, l, M, D, K):
        M, D, K = (np.ascontiguousarray(a, dtype=np.float64) for a in (M, D, K))
        _check(lib().fdg_set_operator_mapped(self._h, l, _ptr(M), _ptr(D), _ptr(K)))

    def set_operator_fields(self, coef):
        coef = np.ascontiguousarray(coef, dtype=np.float64).ravel()
        _check(lib().fdg_set_operator_fields(self._h, _ptr(coef)))

    def _vec(self, t):
        """Pointer of a batch*N vector of this context."""
        return _dev_ptr(t, self.N * self.batch, self.device)

    def apply_prec(self, b, s):
        _check(lib().fdg_apply_prec(self._h, self._vec(b), self._vec(s)))

    def apply_prec_noalloc(self, b, s):
        """fdg_apply_prec_noalloc: the same result, intermediates in the library's static
        device scratch array (nothing allocated)."""
        _check(lib().fdg_apply_prec_noalloc(self._h, self._vec(b), self._vec(s)))

    def matvec(self, x, y):
        _check(lib().fdg_matvec(self._h, self._vec(x), self._vec(y)))

    def solve(self, b, x, rtol=1e-8, restart=30, maxit=1000, flags=0):
        info = fdg_info()
        st = _lib.fdg_solve(self._h, self._vec(b), self._vec(x), rtol, restart, maxit, flags, ctypes.byref(info))
        if st != FDG_OK and st != FDG_NOT_CONVERGED:
            _check(st)
        return {"iterations": info.iterations, "restarts": info.restarts, "converged": info.converged,
                "breakdown": info.breakdown, "rel_res_est": info.rel_res_est, "rel_res_true": info.rel_res_true,
                "ms_total": info.ms_total, "t_apply_ms": info.t_apply_ms, "t_matvec_ms": info.t_matvec_ms,
                "t_orth_ms": info.t_orth_ms, "t_host_ms": info.t_host_ms}

    def operator_bytes(self):
        """Bytes of operator data one matvec reads (x and y excluded)."""
        return int(lib().fdg_operator_bytes(self._h))

    def device_bytes(self):
        """(held, workspace): device bytes the context holds, and the releasable part."""
        held, ws = ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().fdg_ctx_bytes(self._h, ctypes.byref(held), ctypes.byref(ws)))
        return int(held.value), int(ws.value)

    def release_workspace(self):
        """Frees the solve/apply workspace after the stream drains; allocated again on use."""
        _check(lib().fdg_release_workspace(self._h))
        self._ws = None

    def attach_workspace(self, buf, restart=30):
        """Carves the solve/apply workspace from `buf` (a contiguous uint8 device tensor of at
        least workspace_bytes(d, n, batch, restart) bytes, kept referenced while attached;
        contexts sharing it must not run calls that overlap in time); None detaches."""
        if buf is None:
            _check(lib().fdg_attach_workspace(self._h, None, 0, 0))
            self._ws = None
            return
        import torch
        if not isinstance(buf, torch.Tensor) or buf.dtype != torch.uint8 or not buf.is_contiguous():
            raise ValueError("expected a contiguous uint8 tensor")
        if not buf.is_cuda or buf.device.index != self.device:
            raise ValueError(f"workspace must be on cuda:{self.device}")
        need = workspace_bytes(self.d, self.n, self.batch, restart)
        if buf.numel() < need:
            raise ValueError(f"workspace of {buf.numel()} bytes, {need} needed")
        _check(lib().fdg_attach_workspace(self._h, ctypes.c_void_p(buf.data_ptr()), buf.numel(), restart))
        self._ws = buf

    def bicgstab(self, b, x, rtol=1e-8, maxit=1000, flags=0):
        """Preconditioned BiCGStab; "iterations" is the paper's count (k or k + 0.5)."""
        info = fdg_info()
        st = _lib.fdg_bicgstab(self._h, self._vec(b), self._vec(x), rtol, maxit, flags, ctypes.byref(info))
        if st != FDG_OK and st != FDG_NOT_CONVERGED:
            _check(st)
        return {"iterations": info.half_steps / 2.0, "full_iterations": info.iterations,
                "half_steps": info.half_steps, "converged": info.converged, "breakdown": info.breakdown,
                "rel_res_est": info.rel_res_est, "rel_res_true": info.rel_res_true, "ms_total": info.ms_total}

    def timer_enable(self, kernel, on=True):
        _check(lib().fdg_timer_enable(self._h, kernel, int(on)))

    def timer_read(self, kernel):
        cnt = ctypes.c_int64(); ms = ctypes.c_double()
        _check(lib().fdg_timer_read(self._h, kernel, ctypes.byref(cnt), ctypes.byref(ms)))
        return cnt.value, ms.value


class Server:
    """Request server of the C ABI (fdg_server_*): continuous batching of solves."""

    def __init__(self, max_slots, restart=30, lanes=4, arena_bytes=8 << 30):
        h = ctypes.c_void_p()
        _check(lib().fdg_server_create(ctypes.byref(h), max_slots, restart, lanes, arena_bytes))
        self._h = h
        self.restart = restart
        self._cap = max_slots
        self._done = (fdg_done * max_slots)()
        # b and x of every request in flight, by tag: the server writes x (and reads b)
        # until the request completes, so their memory must not return to torch's allocator
        self._held = {}

    def close(self):
        if self._h:
            lib().fdg_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run_bytes(self, ctx):
        return int(lib().fdg_server_run_bytes(ctx._h, self.restart))

    def admit(self, ctx, b, x, rtol=1e-8, maxit=1000, flags=0, tag=0):
        """True when admitted, False when no slot or arena space is free (FDG_EFULL)."""
        if ctx.batch != 1:
            raise ValueError("served requests need a context with batch 1")
        st = lib().fdg_server_admit(self._h, ctx._h, ctx._vec(b), ctx._vec(x), rtol, maxit, flags, tag)
        _check(st, allow=(FDG_OK, FDG_EFULL))
        if st == FDG_OK:
            self._held.setdefault(tag, []).append((b, x))
        return st == FDG_OK

    def step(self, wait_us=0):
        """Advances ready lanes; returns [(tag, status, info dict)] of completed requests."""
        nd = ctypes.c_int()
        _check(lib().fdg_server_step(self._h, int(wait_us), self._done, self._cap, ctypes.byref(nd)))
        out = []
        for k in range(nd.value):
            d = self._done[k]
            held = self._held.get(d.tag)
            if held:
                held.pop(0)
                if not held:
                    del self._held[d.tag]
            out.append((d.tag, d.status, {f: getattr(d.info, f) for f, _ in fdg_info._fields_}))
        return out

    def pending(self):
        return int(lib().fdg_server_pending(self._h))

    def stats(self):
        v = [ctypes.c_int64() for _ in range(4)]
        _check(lib().fdg_server_stats(self._h, *[ctypes.byref(a) for a in v]))
        return dict(zip(("services", "groups", "grouped_runs", "max_group"), (a.value for a in v)))


def unit_context(d, n, M, K, U, V, lam, batch=1, stream=None, prec=PREC_FP64):
    """Context of the unit-domain problem from given 1D factors (operator eq. 2.7 / 2.9 and
    its FD preconditioner, the same factors in every direction)."""
    ctx = Context(d, n, batch=batch, stream=stream)
    for l in range(d):
        ctx.set_prec_factors(l, U, V, lam)
        ctx.set_operator_kron(l, M, K)
    ctx.set_precision(prec)
    return ctx


def unit_problem(d, p, n, batch=1, stream=None, prec=PREC_FP64):
    """Context for the unit-domain collocation problem: operator (eq. 2.7 / 2.9) and its FD
    preconditioner, all factors built by the library's host setup."""
    M, K, D1, tau = colloc_factors(p, n)
    U, V, lam, _ = factor_pencil(K, M, want_cond=False)
    ctx = Context(d, n, batch=batch, stream=stream)
    for l in range(d):
        ctx.set_prec_factors(l, U, V, lam)
        ctx.set_operator_kron(l, M, K)
    ctx.set_precision(prec)
    ctx.tau = tau
    return ctx


def deformed_problem(p, n, amp=0.1, band=False, stream=None, prec=PREC_FP64):
    """Context for the deformed-cube collocation problem (CSR operator) preconditioned by the
    unit-cube FD solve."""
    M, K, D1, tau = colloc_factors(p, n)
    U, V, lam, _ = factor_pencil(K, M, want_cond=False)
    ctx = Context(3, n, stream=stream)
    for l in range(3):
        ctx.set_prec_factors(l, U, V, lam)
    rowptr, col, val = deformed_csr(p, n, amp, band)
    ctx.set_operator_csr(rowptr, col, val)
    ctx.set_precision(prec)
    ctx.tau = tau
    ctx.nnz = len(col)
    return ctx


def mapped_problem(p, n, amp=0.1, stream=None, prec=PREC_FP64):
    """Context for the deformed-cube collocation problem with the operator applied
    matrix-free (1D factors and coefficient fields), preconditioned by the unit-cube FD
    solve."""
    M, K, D1, tau = colloc_factors(p, n)
    U, V, lam, _ = factor_pencil(K, M, want_cond=False)
    ctx = Context(3, n, stream=stream)
    for l in range(3):
        ctx.set_prec_factors(l, U, V, lam)
        ctx.set_operator_mapped(l, M, D1, K)
    ctx.set_operator_fields(deformed_coefficients(p, n, amp))
    ctx.set_precision(prec)
    ctx.tau = tau
    return ctx


def galerkin_problem(p, n, amp=0.0, wind=None, beta=0.0, wind_prec=True, stream=None, prec=PREC_FP64):
    """Context for the Galerkin convection-diffusion problem on the deformed cube (CSR
    operator, Sec. 3.2).  The preconditioner is the unit-cube Galerkin discretization: with
    wind_prec and a wind (c_1, c_2, c_3), direction l uses K_l + H_l for the univariate
    wind c_l (1 + z) (eq. 3.9, nonsymmetric FD); otherwise the wind is dropped (eq. 3.7,
    symmetric FD with V = U).  Pencils with complex eigenvalues use the block form of D
    (FP64 preconditioner only)."""
    ctx = Context(3, n, stream=stream)
    for l in range(3):
        cl = 0.0 if wind is None else float(wind[l])
        M, K, H = galerkin_factors(p, n, cl, cl)
        if wind_prec and cl != 0.0:
            # complex eigenvalue pairs (strong wind, coarse mesh) take the 2 x 2 block form
            U, V, lam, mu, _ = factor_pencil_blocks(K + H, M)
            ctx.set_prec_factors_blocks(l, U, V, lam, mu)
        else:
            U, lam = factor_pencil_sym(K, M)
            ctx.set_prec_factors_sym(l, U, lam)
    rowptr, col, val = galerkin_csr(p, n, amp, wind, beta)
    ctx.set_operator_csr(rowptr, col, val)
    ctx.set_precision(prec)
    ctx.nnz = len(col)
    return ctx
